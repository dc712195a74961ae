// Learned equilibrium of one site per lane, evaluated a wavefront at a time
// on the matrix cores (see mlp_common.hpp for the fragment layout).
//
// For shifted populations g (37 per lane):
//   z = g / w, standardised -> MLP 37-128-128-37 (GELU, BF16 operands,
//   FP32 accumulation) -> y = mean_y + sd_y * o -> d = w y;
//   g_hat = P(g) + d - P(d)   (P: the conserved part; mass, momentum and
//   energy of g_hat are those of g);
//   residual = largest deviation of g_hat's stress and heat flux from the
//   equilibrium values of (rho, u, T); the site falls back to the plain
//   equilibrium when the residual exceeds the threshold or (rho, |u|, T)
//   leaves the training box.
// The 64 sites of a wavefront go through the network in two halves of 32
// (two 16-row tiles), with inputs and hidden activations staged in a
// per-wavefront LDS area; weights are read as fragments from global memory.
#pragma once

#include "mlp_common.hpp"

namespace d2q37 {
namespace mlp {

constexpr int LDX = 72;    // row stride (elements) of the staged inputs
constexpr int LDH = 136;   // row stride of the staged hidden activations
constexpr int WAVE_LDS_BYTES = (32 * LDX + 32 * LDH) * 2;  // 13312

// Orders LDS traffic between the lanes of one wavefront.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Network outputs o[37] (standardised) for each lane's inputs. Every lane of
// the wavefront must call it; inactive lanes pass any finite g.
__device__ inline void network_outputs(const float (&g)[Q], const Net& net, uint16_t* lds, float (&o)[Q])
{
    const int lane = lane_id();
    uint16_t* X = lds;
    uint16_t* H = lds + 32 * LDX;
    float* O = (float*)H;
    const float* b1 = net.params + OFF_B1;
    const float* b2 = net.params + OFF_B2;
    const float* b3 = net.params + OFF_B3;
    const int col = lane & 15, quad = lane >> 4;

    for (int half = 0; half < 2; ++half) {
        if ((lane >> 5) == half) {
            uint16_t* row = X + (lane & 31) * LDX;
#pragma unroll
            for (int f = 0; f < Q; ++f) {
                const float z = g[f] * (float)(1.0 / weight(f));
                row[f] = bf16_bits((z - net.norm[f]) * net.norm[64 + f]);
            }
#pragma unroll
            for (int f = Q; f < KIN; ++f) row[f] = 0;
        }
        wave_sync();

        // layer 1: [32 x 64] x [64 x 128]
        f32x4 acc[2][8];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 a0 = frag_im(X, LDX, 0, ks * 32), a1 = frag_im(X, LDX, 16, ks * 32);
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const bf16x8 b = frag_im(net.W1b, KIN, nt * 16, ks * 32);
                acc[0][nt] = mfma(a0, b, acc[0][nt]);
                acc[1][nt] = mfma(a1, b, acc[1][nt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const int h = nt * 16 + col;
                const float bias = b1[h];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    H[(mt * 16 + 4 * quad + i) * LDH + h] = bf16_bits(gelu(acc[mt][nt][i] + bias));
            }
        wave_sync();

        // layer 2: [32 x 128] x [128 x 128], in place on H
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 a0 = frag_im(H, LDH, 0, ks * 32), a1 = frag_im(H, LDH, 16, ks * 32);
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const bf16x8 b = frag_im(net.W2b, HID, nt * 16, ks * 32);
                acc[0][nt] = mfma(a0, b, acc[0][nt]);
                acc[1][nt] = mfma(a1, b, acc[1][nt]);
            }
        }
        wave_sync();
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const int h = nt * 16 + col;
                const float bias = b2[h];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    H[(mt * 16 + 4 * quad + i) * LDH + h] = bf16_bits(gelu(acc[mt][nt][i] + bias));
            }
        wave_sync();

        // layer 3: [32 x 128] x [128 x 48]
        f32x4 acc3[2][3];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 3; ++nt) acc3[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 a0 = frag_im(H, LDH, 0, ks * 32), a1 = frag_im(H, LDH, 16, ks * 32);
#pragma unroll
            for (int nt = 0; nt < 3; ++nt) {
                const bf16x8 b = frag_im(net.W3b, HID, nt * 16, ks * 32);
                acc3[0][nt] = mfma(a0, b, acc3[0][nt]);
                acc3[1][nt] = mfma(a1, b, acc3[1][nt]);
            }
        }
        wave_sync();
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 3; ++nt) {
                const int oc = nt * 16 + col;
                const float bias = oc < Q ? b3[oc] : 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) O[(mt * 16 + 4 * quad + i) * NOUT + oc] = acc3[mt][nt][i] + bias;
            }
        wave_sync();
        if ((lane >> 5) == half) {
            const float* row = O + (lane & 31) * NOUT;
#pragma unroll
            for (int f = 0; f < Q; ++f) o[f] = row[f];
        }
        wave_sync();
    }
}

struct Verdict {
    bool fallback;
    float residual;
};

// g_hat (learned, projected) and the fallback verdict of each lane's site.
__device__ inline Verdict learned_equilibrium(const float (&g)[Q], const Net& net, uint16_t* lds, float threshold,
                                              float (&ghat)[Q])
{
    float o[Q];
    network_outputs(g, net, lds, o);
    float d[Q];
#pragma unroll
    for (int f = 0; f < Q; ++f) d[f] = mulk(__builtin_fmaf(net.norm[192 + f], o[f], net.norm[128 + f]), weight(f));
    const Conserved mg = conserved_moments(g);
    const Conserved md = conserved_moments(d);
    const ConservedCoef k = conserved_coef(mg.m0 - md.m0, mg.mx - md.mx, mg.my - md.my, mg.mE - md.mE);
#pragma unroll
    for (int f = 0; f < Q; ++f) ghat[f] = d[f] + conserved_value(f, k);

    // residual against the equilibrium stress and heat flux of (rho, u, T)
    const float rho = 1.0f + mg.m0;
    const float ux = mg.mx / rho, uy = mg.my / rho;
    const float u2 = ux * ux + uy * uy;
    const float T = 1.0f + (mg.mE - rho * u2) / (2.0f * rho);
    float sxy = 0.f, snn = 0.f, sqx = 0.f, sqy = 0.f;  // lattice units
#pragma unroll
    for (int f = 0; f < Q; ++f) {
        if (CX[f] * CY[f] != 0) sxy = __builtin_fmaf((float)(CX[f] * CY[f]), ghat[f], sxy);
        if (CX[f] * CX[f] - CY[f] * CY[f] != 0)
            snn = __builtin_fmaf((float)(CX[f] * CX[f] - CY[f] * CY[f]), ghat[f], snn);
        if (CX[f] != 0) sqx = __builtin_fmaf((float)(CX[f] * c2_of(f)), ghat[f], sqx);
        if (CY[f] != 0) sqy = __builtin_fmaf((float)(CY[f] * c2_of(f)), ghat[f], sqy);
    }
    const float q4 = u2 + 4.0f * T;
    const float r1 = fabsf(mulk(sxy, R2) - rho * ux * uy);
    const float r2 = fabsf(mulk(snn, R2) - rho * (ux * ux - uy * uy));
    const float r3 = fabsf(mulk(sqx, R * R2) - rho * ux * q4);
    const float r4 = fabsf(mulk(sqy, R * R2) - rho * uy * q4);
    Verdict v;
    v.residual = fmaxf(fmaxf(r1, r2), fmaxf(r3, r4));
    const bool in_box = rho >= 0.9f && rho <= 1.1f && u2 <= 0.01f && T >= 0.9f && T <= 1.1f;
    v.fallback = !in_box || !(v.residual <= threshold);
    return v;
}

}  // namespace mlp
}  // namespace d2q37
