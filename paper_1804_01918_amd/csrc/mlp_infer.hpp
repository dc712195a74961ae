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
// The 64 sites of a wavefront go through the network in two halves of 32.
// Layers are computed transposed (hidden x sites) and chained in registers
// (see chain_hidden in mlp_common.hpp); only the inputs (to bring each
// site's 37 values into fragment order) and the outputs (to return each
// site's 37 outputs to its lane) pass through a per-wavefront LDS area.
#pragma once

#include "mlp_common.hpp"

namespace d2q37 {
namespace mlp {

constexpr int LDX = 80;    // row stride (bf16) of the staged inputs of a wavefront's 64 sites
constexpr int LDH = 136;   // row stride of staged hidden activations (training)
constexpr int LDO = 40;    // row stride (floats) of the staged outputs: same bytes as an input row
constexpr int WAVE_LDS_BYTES = 64 * LDX * 2;  // 10240

// Orders LDS traffic between the lanes of one wavefront.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline float4 load4(const float* p) { return *(const float4*)p; }

// Standardised BF16 input of population p (value g) into the lane's row.
__device__ inline void stage_input(uint16_t* X, const Net& net, int p, float g)
{
    const float z = g * (float)(1.0 / weight(p));
    X[lane_id() * LDX + p] = bf16_bits((z - net.norm[p]) * net.norm[64 + p]);
}
__device__ inline void stage_padding(uint16_t* X)
{
#pragma unroll
    for (int f = Q; f < LDX; ++f) X[lane_id() * LDX + f] = 0;
}

// Network outputs of the wavefront's 64 sites. X holds the staged inputs
// (row per site); on return the same rows hold the standardised outputs as
// FP32, out[site * LDO + o] for o < 37. Every lane must call it.
__device__ inline void network_outputs(const Net& net, uint16_t* X)
{
    const int lane = lane_id(), col = lane & 15, quad = lane >> 4;
    const float* b1 = net.params + OFF_B1;
    const float* b2 = net.params + OFF_B2;
    const float* b3 = net.params + OFF_B3;
    wave_sync();

#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        uint16_t* Xh = X + half * 32 * LDX;

        // layer 1: H1^T (128 x 32) = W1 (128 x 64) X^T (64 x 32)
        f32x4 acc[8][2];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt][0] = acc[mt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            __builtin_amdgcn_sched_barrier(0);  // one k block of weight fragments in flight
            const bf16x8 x0 = frag_im(Xh, LDX, 0, ks * 32), x1 = frag_im(Xh, LDX, 16, ks * 32);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt) {
                const bf16x8 a = frag_im(net.W1b, net.ld1, mt * 16, ks * 32);
                acc[mt][0] = mfma(a, x0, acc[mt][0]);
                acc[mt][1] = mfma(a, x1, acc[mt][1]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // bias, GELU, BF16 into the B fragments of the next layer
        bf16x8 hb[4][2];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const float4 lo = load4(b1 + 32 * kb + 4 * quad), hi = load4(b1 + 32 * kb + 16 + 4 * quad);
            const float bl[4] = {lo.x, lo.y, lo.z, lo.w}, bh[4] = {hi.x, hi.y, hi.z, hi.w};
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    hb[kb][nt][j] = __builtin_bit_cast(__bf16, bf16_bits(gelu_fast(acc[2 * kb][nt][j] + bl[j])));
                    hb[kb][nt][4 + j] = __builtin_bit_cast(__bf16, bf16_bits(gelu_fast(acc[2 * kb + 1][nt][j] + bh[j])));
                }
        }

        // layer 2: H2^T = W2 H1^T (weight columns in chained order)
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt][0] = acc[mt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt) {
                const bf16x8 a = frag_im(net.W2p, net.ld23, mt * 16, kb * 32);
                acc[mt][0] = mfma(a, hb[kb][0], acc[mt][0]);
                acc[mt][1] = mfma(a, hb[kb][1], acc[mt][1]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const float4 lo = load4(b2 + 32 * kb + 4 * quad), hi = load4(b2 + 32 * kb + 16 + 4 * quad);
            const float bl[4] = {lo.x, lo.y, lo.z, lo.w}, bh[4] = {hi.x, hi.y, hi.z, hi.w};
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    hb[kb][nt][j] = __builtin_bit_cast(__bf16, bf16_bits(gelu_fast(acc[2 * kb][nt][j] + bl[j])));
                    hb[kb][nt][4 + j] = __builtin_bit_cast(__bf16, bf16_bits(gelu_fast(acc[2 * kb + 1][nt][j] + bh[j])));
                }
        }

        // layer 3: O^T (48 x 32) = W3 H2^T
        f32x4 acc3[3][2];
#pragma unroll
        for (int mt = 0; mt < 3; ++mt) acc3[mt][0] = acc3[mt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mt = 0; mt < 3; ++mt) {
                const bf16x8 a = frag_im(net.W3p, net.ld23, mt * 16, kb * 32);
                acc3[mt][0] = mfma(a, hb[kb][0], acc3[mt][0]);
                acc3[mt][1] = mfma(a, hb[kb][1], acc3[mt][1]);
            }
        }
        wave_sync();  // the half's input rows are dead before its outputs overwrite them
        float* O = (float*)Xh;
#pragma unroll
        for (int mt = 0; mt < 3; ++mt) {
            const int o = mt * 16 + 4 * quad;
            if (o < LDO) {
                float bb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) bb[i] = (o + i) < Q ? b3[o + i] : 0.f;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int site = 16 * nt + col;
                    *(float4*)(O + site * LDO + o) = float4{acc3[mt][nt][0] + bb[0], acc3[mt][nt][1] + bb[1],
                                                           acc3[mt][nt][2] + bb[2], acc3[mt][nt][3] + bb[3]};
                }
            }
        }
    }
    wave_sync();
}

// LDS copy of the inference weights, rows padded by 16 bytes so that the 16
// rows of a fragment fall on different banks.
constexpr int LDW1 = KIN + 8;
constexpr int LDW23 = HID + 8;
struct SharedWeights {
    uint16_t W1[HID * LDW1];
    uint16_t W2[HID * LDW23];
    uint16_t W3[NOUT * LDW23];
};

// Copy the BF16 inference weights of `net` into LDS (all threads of the
// workgroup; the caller synchronises) and return the view that reads them.
template <int NTHREADS>
__device__ inline Net share_weights(const Net& net, SharedWeights& S)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < HID * KIN / 8; i += NTHREADS) {
        const int r = i / (KIN / 8), c = (i % (KIN / 8)) * 8;
        *(uint4*)(S.W1 + r * LDW1 + c) = *(const uint4*)(net.W1b + r * KIN + c);
    }
    for (int i = tid; i < HID * HID / 8; i += NTHREADS) {
        const int r = i / (HID / 8), c = (i % (HID / 8)) * 8;
        *(uint4*)(S.W2 + r * LDW23 + c) = *(const uint4*)(net.W2p + r * HID + c);
    }
    for (int i = tid; i < NOUT * HID / 8; i += NTHREADS) {
        const int r = i / (HID / 8), c = (i % (HID / 8)) * 8;
        *(uint4*)(S.W3 + r * LDW23 + c) = *(const uint4*)(net.W3p + r * HID + c);
    }
    Net v = net;
    v.W1b = S.W1;
    v.W2p = S.W2;
    v.W3p = S.W3;
    v.ld1 = LDW1;
    v.ld23 = LDW23;
    return v;
}

struct Verdict {
    bool fallback;
    float residual;
};

// The learned equilibrium of a lane's site, evaluated on demand from the
// staged network outputs: g_hat_p = d_p + P(g - d)_p, d_p = w_p (mean_y +
// sd_y o_p).
struct Learned {
    const float* row;
    ConservedCoef k;
    Verdict verdict;
};

__device__ inline float learned_d(const Net& net, const float* row, int p)
{
    return mulk(__builtin_fmaf(net.norm[192 + p], row[p], net.norm[128 + p]), weight(p));
}
__device__ inline float learned_value(const Learned& L, const Net& net, int p)
{
    return learned_d(net, L.row, p) + conserved_value(p, L.k);
}

// Projection coefficients and fallback verdict of each lane's site from its
// populations g and the network outputs staged by network_outputs (residual
// against the equilibrium stress and heat flux of (rho, u, T); training box
// on rho, |u|, T).
__device__ inline Learned learned_equilibrium(const float (&g)[Q], const Net& net, const uint16_t* X, float threshold)
{
    Learned L;
    L.row = (const float*)X + lane_id() * LDO;
    float d0 = 0.f, dx = 0.f, dy = 0.f, de = 0.f;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float d = learned_d(net, L.row, p);
        d0 += d;
        if (CX[p] != 0) dx = __builtin_fmaf((float)CX[p], d, dx);
        if (CY[p] != 0) dy = __builtin_fmaf((float)CY[p], d, dy);
        if (c2_of(p) != 0) de = __builtin_fmaf((float)c2_of(p), d, de);
    }
    const Conserved mg = conserved_moments(g);
    const float md0 = d0, mdx = mulk(dx, R), mdy = mulk(dy, R), mdE = mulk(de, R2) - 2.0f * d0;
    L.k = conserved_coef(mg.m0 - md0, mg.mx - mdx, mg.my - mdy, mg.mE - mdE);

    const float rho = 1.0f + mg.m0;
    const float ux = mg.mx / rho, uy = mg.my / rho;
    const float u2 = ux * ux + uy * uy;
    const float T = 1.0f + (mg.mE - rho * u2) / (2.0f * rho);
    float sxy = 0.f, snn = 0.f, sqx = 0.f, sqy = 0.f;  // lattice units
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float gh = learned_value(L, net, p);
        if (CX[p] * CY[p] != 0) sxy = __builtin_fmaf((float)(CX[p] * CY[p]), gh, sxy);
        if (CX[p] * CX[p] - CY[p] * CY[p] != 0)
            snn = __builtin_fmaf((float)(CX[p] * CX[p] - CY[p] * CY[p]), gh, snn);
        if (CX[p] != 0) sqx = __builtin_fmaf((float)(CX[p] * c2_of(p)), gh, sqx);
        if (CY[p] != 0) sqy = __builtin_fmaf((float)(CY[p] * c2_of(p)), gh, sqy);
    }
    const float q4 = u2 + 4.0f * T;
    const float r1 = fabsf(mulk(sxy, R2) - rho * ux * uy);
    const float r2 = fabsf(mulk(snn, R2) - rho * (ux * ux - uy * uy));
    const float r3 = fabsf(mulk(sqx, R * R2) - rho * ux * q4);
    const float r4 = fabsf(mulk(sqy, R * R2) - rho * uy * q4);
    L.verdict.residual = fmaxf(fmaxf(r1, r2), fmaxf(r3, r4));
    const bool in_box = rho >= 0.9f && rho <= 1.1f && u2 <= 0.01f && T >= 0.9f && T <= 1.1f;
    L.verdict.fallback = !in_box || !(L.verdict.residual <= threshold);
    return L;
}

}  // namespace mlp
}  // namespace d2q37
