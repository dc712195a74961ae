// Learned collide: training pairs, network initialisation, standardisation,
// forward/backward and Adam on the gfx950 matrix cores, and evaluation of
// the learned equilibrium (C ABI declared in include/lb.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>

#include "../../include/lb.h"
#include "lb_mlp_state.hpp"
#include "mlp_infer.hpp"

using namespace d2q37;
using namespace d2q37::mlp;

namespace {

constexpr int TB = 256;

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC11) --------------------------
struct Ctr {
    uint32_t v[4];
};
__device__ inline Ctr philox(Ctr c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c.v[0]), lo0 = M0 * c.v[0];
        const uint32_t hi1 = __umulhi(M1, c.v[2]), lo1 = M1 * c.v[2];
        c = Ctr{{hi1 ^ c.v[1] ^ k0, lo1, hi0 ^ c.v[3] ^ k1, lo0}};
        k0 += W0;
        k1 += W1;
    }
    return c;
}
// Top 23 bits as an odd multiple of 2^-24: exact in FP32, inside (0, 1).
__device__ inline float unit_open(uint32_t x) { return (float)((x >> 9) * 2u + 1u) * 5.9604644775390625e-8f; }

// ---- training pairs -------------------------------------------------------------
// Pair k: key (seed lo, seed hi), counters (k lo, k hi, j, 0) for j = 0..10:
// rho = 0.9 + 0.2 U0, u = 0.1 sqrt(U1) (cos, sin)(2 pi U2), T = 0.9 + 0.2 U3,
// normals by Box-Muller from (U[4 + 2q], U[5 + 2q]); pre = g_eq + 1e-3 w n,
// post = the plain FP32 collide of pre.
__global__ __launch_bounds__(TB) void k_pairgen(float* __restrict__ pre, float* __restrict__ post, int64_t n,
                                                uint32_t key0, uint32_t key1, float omega)
{
    const int64_t k = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (k >= n) return;
    uint32_t w[44];
#pragma unroll
    for (int j = 0; j < 11; ++j) {
        const Ctr r = philox(Ctr{{(uint32_t)k, (uint32_t)((uint64_t)k >> 32), (uint32_t)j, 0u}}, key0, key1);
#pragma unroll
        for (int q = 0; q < 4; ++q) w[4 * j + q] = r.v[q];
    }
    const float rho = 0.9f + 0.2f * unit_open(w[0]);
    const float rad = 0.1f * sqrtf(unit_open(w[1]));
    float sn, cs;
    sincosf(6.28318530717958647692f * unit_open(w[2]), &sn, &cs);
    const float ux = rad * cs, uy = rad * sn;
    const float T = 0.9f + 0.2f * unit_open(w[3]);
    float nrm[38];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const float mag = sqrtf(-2.0f * logf(unit_open(w[4 + 2 * q])));
        float s2, c2;
        sincosf(6.28318530717958647692f * unit_open(w[5 + 2 * q]), &s2, &c2);
        nrm[2 * q] = mag * c2;
        nrm[2 * q + 1] = mag * s2;
    }
    Macro<float> m;
    m.rho = rho;
    m.drho = rho - 1.0f;
    m.Ux = mulk(ux, R);
    m.Uy = mulk(uy, R);
    m.u2 = ux * ux + uy * uy;
    m.t = T - 1.0f;
    float zero[Q], g[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) zero[p] = 0.0f;
    relax_emit<float, true>(zero, m, 1.0f, 0.0f, [&](int p, float v) { g[p] = v; });
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        g[p] = __builtin_fmaf(mulk(1e-3f, weight(p)), nrm[p], g[p]);
        pre[k * Q + p] = g[p];
    }
    collide_site<PrecF32S, true>(g, omega, [&](int p, float v) { post[k * Q + p] = v; });
}

// ---- parameters -------------------------------------------------------------------
// Xavier-uniform weights from Philox counter (i, 0, 0xFFFFFFFF, 0), zero biases.
__global__ __launch_bounds__(TB) void k_mlp_init(float* __restrict__ params, uint32_t key0, uint32_t key1)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= NPARAM) return;
    int fan = 0;
    if (i < OFF_B1) fan = HID + Q;
    else if (i >= OFF_W2 && i < OFF_B2) fan = HID + HID;
    else if (i >= OFF_W3 && i < OFF_B3) fan = Q + HID;
    if (fan == 0) {
        params[i] = 0.0f;
        return;
    }
    const Ctr r = philox(Ctr{{(uint32_t)i, 0u, 0xFFFFFFFFu, 0u}}, key0, key1);
    const double u = ((double)(r.v[0] >> 9) * 2.0 + 1.0) * 5.9604644775390625e-8;
    const double a = sqrt(6.0 / (double)fan);
    params[i] = (float)(a * (2.0 * u - 1.0));
}

// Operand copies of the weights, zero padding included: BF16 (training,
// and the first layer of inference) and the binary16 W2p, W3p of inference.
__global__ __launch_bounds__(TB) void k_mlp_pack(const float* __restrict__ params, uint16_t* __restrict__ W1b,
                                                 uint16_t* __restrict__ W2b, uint16_t* __restrict__ W3b,
                                                 uint16_t* __restrict__ W2t, uint16_t* __restrict__ W3t,
                                                 uint16_t* __restrict__ W2p, uint16_t* __restrict__ W3p)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i < HID * HID) {  // W2p[h2][slot]
        const int a = i / HID, slot = i % HID;
        W2p[i] = f16_bits(params[OFF_W2 + a * HID + chain_hidden(slot)]);
    }
    if (i < NOUT * HID) {  // W3p[o][slot]
        const int o = i / HID, slot = i % HID;
        W3p[i] = o < Q ? f16_bits(params[OFF_W3 + o * HID + chain_hidden(slot)]) : 0;
    }
    if (i < HID * KIN) {  // W1b[h][f], W3t[h][o]
        const int h = i / KIN, f = i % KIN;
        W1b[i] = f < Q ? bf16_bits(params[OFF_W1 + h * Q + f]) : 0;
        W3t[i] = f < Q ? bf16_bits(params[OFF_W3 + f * HID + h]) : 0;
    }
    if (i < HID * HID) {  // W2b[h2][h1], W2t[h1][h2]
        const int a = i / HID, b = i % HID;
        W2b[i] = bf16_bits(params[OFF_W2 + a * HID + b]);
        W2t[i] = bf16_bits(params[OFF_W2 + b * HID + a]);
    }
    if (i < NOUT * HID) {  // W3b[o][h]
        const int o = i / HID, h = i % HID;
        W3b[i] = o < Q ? bf16_bits(params[OFF_W3 + o * HID + h]) : 0;
    }
}

// The FP8 form's scaled copies (see Net), one workgroup: the exponent aw
// puts max |W2| in [128, 256) (max |W2| = f 2^e, f in [0.5, 1): aw = 8 - e).
__global__ __launch_bounds__(TB) void k_mlp_pack_fp8(const float* __restrict__ params, uint16_t* __restrict__ W1s,
                                                     uint8_t* __restrict__ W2q, uint16_t* __restrict__ W3s,
                                                     float* __restrict__ b1s, float* __restrict__ b2s,
                                                     float* __restrict__ gk2)
{
    __shared__ float red[TB];
    const int tid = threadIdx.x;
    float mx = 0.0f;
    for (int i = tid; i < HID * HID; i += TB) mx = fmaxf(mx, fabsf(params[OFF_W2 + i]));
    red[tid] = mx;
    __syncthreads();
    for (int half = TB / 2; half > 0; half >>= 1) {
        if (tid < half) red[tid] = fmaxf(red[tid], red[tid + half]);
        __syncthreads();
    }
    int e = 0;
    frexpf(red[0] > 0.0f ? red[0] : 1.0f, &e);
    const int aw = 8 - e;
    const float sw = ldexpf(1.0f, aw);
    const float s3 = ldexpf(1.0f, -(aw + 4));  // 1 / (2^aw FP8_ACT_SCALE)
    for (int i = tid; i < HID * HID; i += TB) {  // W2q[h2][slot]
        const int a = i / HID, slot = i % HID;
        W2q[i] = (uint8_t)(pack_fp8<false>(params[OFF_W2 + a * HID + chain_hidden(slot)] * sw, 0.0f, 0u) & 0xFFu);
    }
    for (int i = tid; i < HID * KIN; i += TB) {  // W1s[h][f]
        const int h = i / KIN, f = i % KIN;
        W1s[i] = f < Q ? bf16_bits(FP8_ACT_SCALE * params[OFF_W1 + h * Q + f]) : 0;
    }
    for (int i = tid; i < NOUT * HID; i += TB) {  // W3s[o][slot]
        const int o = i / HID, slot = i % HID;
        W3s[i] = o < Q ? bf16_bits(s3 * params[OFF_W3 + o * HID + chain_hidden(slot)]) : 0;
    }
    for (int i = tid; i < HID; i += TB) {
        b1s[i] = FP8_ACT_SCALE * params[OFF_B1 + i];
        b2s[i] = params[OFF_B2 + i] / s3;
    }
    if (tid == 0) {
        gk2[0] = GELU_K1 * (s3 * s3 * s3);
        gk2[1] = GELU_K2 * s3;
    }
}

// Per-feature sums over the pairs (pass 0: values; pass 1: squared
// deviations from `mean`), FP64, fixed order: block partials then a final sum.
constexpr int STAT_TILE = 128;
__global__ __launch_bounds__(TB) void k_mlp_stats(const float* __restrict__ pre, const float* __restrict__ post,
                                                  int64_t n, float tau, int pass, const double* __restrict__ mean,
                                                  double* __restrict__ partials)
{
    __shared__ float F[STAT_TILE][NSTAT + 1];
    double acc = 0.0;
    const int j = threadIdx.x;
    for (int64_t base = (int64_t)blockIdx.x * STAT_TILE; base < n; base += (int64_t)gridDim.x * STAT_TILE) {
        __syncthreads();
        if (threadIdx.x < STAT_TILE && base + threadIdx.x < n) {
            const int64_t s = base + threadIdx.x;
            float z[Q], y[Q];
            pair_features(pre + s * Q, post + s * Q, tau, z, y);
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                F[threadIdx.x][p] = z[p];
                F[threadIdx.x][Q + p] = y[p];
            }
        }
        __syncthreads();
        if (j < NSTAT) {
            const int cnt = (int)((n - base) < STAT_TILE ? (n - base) : STAT_TILE);
            const double mu = pass ? mean[j] : 0.0;
            for (int s = 0; s < cnt; ++s) {
                const double v = (double)F[s][j] - mu;
                acc += pass ? v * v : v;
            }
        }
    }
    if (j < NSTAT) partials[(int64_t)blockIdx.x * NSTAT + j] = acc;
}

__global__ void k_mlp_stats_final(const double* __restrict__ partials, int nblocks, int64_t n, int pass,
                                  double* __restrict__ mean, float* __restrict__ norm)
{
    const int j = threadIdx.x;
    if (j >= NSTAT) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * NSTAT + j];
    if (pass == 0) {
        mean[j] = s / (double)n;
        return;
    }
    double sd = sqrt(s / (double)n);
    if (!(sd >= 1e-12)) sd = 1.0;
    if (j < Q) {
        norm[j] = (float)mean[j];
        norm[64 + j] = (float)(1.0 / sd);
    } else {
        norm[128 + j - Q] = (float)mean[j];
        norm[192 + j - Q] = (float)sd;
    }
}

// Folded standardisation for inference (Net::fnorm), rounded once from FP64:
// z_std = g a + b with a = 1/(sd_z w), b = -mean_z/sd_z; d = o A + B with
// A = w sd_y, B = w mean_y.
__global__ void k_mlp_fold_norm(const float* __restrict__ norm, float* __restrict__ fnorm)
{
    const int p = threadIdx.x;
    if (p >= 64) return;
    if (p >= Q) {
        fnorm[p] = fnorm[64 + p] = fnorm[128 + p] = fnorm[192 + p] = 0.0f;
        return;
    }
    const double w = weight(p);
    fnorm[p] = (float)((double)norm[64 + p] / w);
    fnorm[64 + p] = (float)(-(double)norm[p] * (double)norm[64 + p]);
    fnorm[128 + p] = (float)(w * (double)norm[192 + p]);
    fnorm[192 + p] = (float)(w * (double)norm[128 + p]);
}

// ---- forward and backward of one training workgroup -------------------------------
// 32 samples, 4 wavefronts. Sample s of step-batch position b is pair
// (a (start + b) + c) mod n. Writes the workgroup's gradient (all NPARAM
// entries) and its share of the loss: sum of squared errors / (B 37).
constexpr int TS = TRAIN_SAMPLES;
struct TrainLds {
    uint16_t X[TS * LDX];
    uint16_t H1[TS * LDH];
    uint16_t H2[TS * LDH];
    uint16_t dOq[TS * LDX];
    uint16_t dA2q[TS * LDH];
    uint16_t dA1q[TS * LDH];
    float A1[TS * HID];
    float A2[TS * HID];
    float Of[TS * NOUT];
    float Yt[TS * Q];
    double red[TB / 64];
};

__global__ __launch_bounds__(TB) void k_mlp_fwdbwd(const float* __restrict__ pre, const float* __restrict__ post,
                                                   int64_t n, int64_t a, int64_t c, int64_t start, int64_t btotal,
                                                   float tau, Net net, float* __restrict__ partials,
                                                   double* __restrict__ lossp)
{
    __shared__ TrainLds L;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int col = lane & 15, quad = lane >> 4;
    float* part = partials + (int64_t)blockIdx.x * NPARAM_PAD;

    // samples: standardised inputs and targets
    if (tid < TS) {
        const int64_t pos = start + (int64_t)blockIdx.x * TS + tid;
        const int64_t idx = (int64_t)(((unsigned __int128)a * (uint64_t)pos + (uint64_t)c) % (uint64_t)n);
        float z[Q], y[Q];
        pair_features(pre + idx * Q, post + idx * Q, tau, z, y);
#pragma unroll
        for (int f = 0; f < Q; ++f) {
            L.X[tid * LDX + f] = bf16_bits((z[f] - net.norm[f]) * net.norm[64 + f]);
            L.Yt[tid * Q + f] = (y[f] - net.norm[128 + f]) / net.norm[192 + f];
        }
        for (int f = Q; f < LDX; ++f) L.X[tid * LDX + f] = 0;
    }
    __syncthreads();

    // layer 1 and 2: 16 tiles (2 sample tiles x 8 hidden tiles); wave w: hidden tiles 2w, 2w+1
    for (int layer = 0; layer < 2; ++layer) {
        const uint16_t* in = layer == 0 ? L.X : L.H1;
        const int ldi = layer == 0 ? LDX : LDH;
        const int ks_n = layer == 0 ? 2 : 4;
        const uint16_t* W = layer == 0 ? net.W1b : net.W2b;
        const int ldw = layer == 0 ? KIN : HID;
        const float* bias = net.params + (layer == 0 ? OFF_B1 : OFF_B2);
        float* A = layer == 0 ? L.A1 : L.A2;
        uint16_t* Hout = layer == 0 ? L.H1 : L.H2;
        for (int t = 0; t < 2; ++t) {
            const int nt = 2 * wave + t;
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < ks_n; ++ks) {
                const bf16x8 b = frag_im(W, ldw, nt * 16, ks * 32);
                acc0 = mfma(frag_im(in, ldi, 0, ks * 32), b, acc0);
                acc1 = mfma(frag_im(in, ldi, 16, ks * 32), b, acc1);
            }
            const int h = nt * 16 + col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int s0 = 4 * quad + i, s1 = 16 + 4 * quad + i;
                const float v0 = acc0[i] + bias[h], v1 = acc1[i] + bias[h];
                A[s0 * HID + h] = v0;
                A[s1 * HID + h] = v1;
                Hout[s0 * LDH + h] = bf16_bits(gelu(v0));
                Hout[s1 * LDH + h] = bf16_bits(gelu(v1));
            }
        }
        __syncthreads();
    }

    // layer 3: 6 tiles (2 sample tiles x 3 output tiles)
    for (int t = wave; t < 6; t += 4) {
        const int mt = t / 3, nt = t % 3;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 4; ++ks) acc = mfma(frag_im(L.H2, LDH, mt * 16, ks * 32), frag_im(net.W3b, HID, nt * 16, ks * 32), acc);
        const int o = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) L.Of[(mt * 16 + 4 * quad + i) * NOUT + o] = o < Q ? acc[i] + net.params[OFF_B3 + o] : 0.f;
    }
    __syncthreads();

    // loss and output gradient dO = 2 (o - y) / (B 37)
    const float scale = (float)(2.0 / ((double)btotal * Q));
    float sq = 0.f;
    for (int e = tid; e < TS * Q; e += TB) {
        const int s = e / Q, o = e % Q;
        const float diff = L.Of[s * NOUT + o] - L.Yt[s * Q + o];
        sq = __builtin_fmaf(diff, diff, sq);
        const float d = diff * scale;
        L.Of[s * NOUT + o] = d;
        L.dOq[s * LDX + o] = bf16_bits(d);
    }
    for (int e = tid; e < TS * (LDX - Q); e += TB) {
        const int s = e / (LDX - Q), o = Q + e % (LDX - Q);
        L.dOq[s * LDX + o] = 0;
    }
    {
        double v = (double)sq;
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) L.red[wave] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < TB / 64; ++w) s += L.red[w];
        lossp[blockIdx.x] = s / ((double)btotal * Q);
    }

    // dH2 = dO W3 -> dA2 = dH2 * gelu'(A2); dW3 = dO^T H2; db3
    for (int t = 0; t < 2; ++t) {
        const int nt = 2 * wave + t;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 b = frag_im(net.W3t, KIN, nt * 16, ks * 32);
            acc0 = mfma(frag_im(L.dOq, LDX, 0, ks * 32), b, acc0);
            acc1 = mfma(frag_im(L.dOq, LDX, 16, ks * 32), b, acc1);
        }
        const int h = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s0 = 4 * quad + i, s1 = 16 + 4 * quad + i;
            const float d0 = acc0[i] * gelu_grad(L.A2[s0 * HID + h]);
            const float d1 = acc1[i] * gelu_grad(L.A2[s1 * HID + h]);
            L.A2[s0 * HID + h] = d0;
            L.A2[s1 * HID + h] = d1;
            L.dA2q[s0 * LDH + h] = bf16_bits(d0);
            L.dA2q[s1 * LDH + h] = bf16_bits(d1);
        }
    }
    for (int t = wave; t < 24; t += 4) {
        const int mt = t / 8, nt = t % 8;  // output rows o (3 tiles) x hidden h (8 tiles)
        const f32x4 acc = mfma(frag_km(L.dOq, LDX, mt * 16, 0), frag_km(L.H2, LDH, nt * 16, 0), f32x4{0.f, 0.f, 0.f, 0.f});
        const int h = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = mt * 16 + 4 * quad + i;
            if (o < Q) part[OFF_W3 + o * HID + h] = acc[i];
        }
    }
    if (tid < Q) {
        float s = 0.f;
        for (int r = 0; r < TS; ++r) s += L.Of[r * NOUT + tid];
        part[OFF_B3 + tid] = s;
    }
    __syncthreads();

    // dH1 = dA2 W2 -> dA1; dW2 = dA2^T H1; db2
    for (int t = 0; t < 2; ++t) {
        const int nt = 2 * wave + t;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x8 b = frag_im(net.W2t, HID, nt * 16, ks * 32);
            acc0 = mfma(frag_im(L.dA2q, LDH, 0, ks * 32), b, acc0);
            acc1 = mfma(frag_im(L.dA2q, LDH, 16, ks * 32), b, acc1);
        }
        const int h = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s0 = 4 * quad + i, s1 = 16 + 4 * quad + i;
            const float d0 = acc0[i] * gelu_grad(L.A1[s0 * HID + h]);
            const float d1 = acc1[i] * gelu_grad(L.A1[s1 * HID + h]);
            L.A1[s0 * HID + h] = d0;
            L.A1[s1 * HID + h] = d1;
            L.dA1q[s0 * LDH + h] = bf16_bits(d0);
            L.dA1q[s1 * LDH + h] = bf16_bits(d1);
        }
    }
    for (int t = wave; t < 64; t += 4) {
        const int mt = t / 8, nt = t % 8;  // h2 tile x h1 tile
        const f32x4 acc = mfma(frag_km(L.dA2q, LDH, mt * 16, 0), frag_km(L.H1, LDH, nt * 16, 0), f32x4{0.f, 0.f, 0.f, 0.f});
        const int h1 = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) part[OFF_W2 + (mt * 16 + 4 * quad + i) * HID + h1] = acc[i];
    }
    if (tid < HID) {
        float s = 0.f;
        for (int r = 0; r < TS; ++r) s += L.A2[r * HID + tid];
        part[OFF_B2 + tid] = s;
    }
    __syncthreads();

    // dW1 = dA1^T X; db1
    for (int t = wave; t < 24; t += 4) {
        const int mt = t / 3, nt = t % 3;  // hidden tile x feature tile
        const f32x4 acc = mfma(frag_km(L.dA1q, LDH, mt * 16, 0), frag_km(L.X, LDX, nt * 16, 0), f32x4{0.f, 0.f, 0.f, 0.f});
        const int f = nt * 16 + col;
        if (f < Q) {
#pragma unroll
            for (int i = 0; i < 4; ++i) part[OFF_W1 + (mt * 16 + 4 * quad + i) * Q + f] = acc[i];
        }
    }
    if (tid < HID) {
        float s = 0.f;
        for (int r = 0; r < TS; ++r) s += L.A1[r * HID + tid];
        part[OFF_B1 + tid] = s;
    }
}

// Sum of the workgroup gradients, then either an Adam step (mode 0;
// parameters and their BF16 copies updated, the step's loss added to
// loss_epoch[epoch]) or a copy of the gradient to grad (mode 1). A workgroup
// takes UPD_PARAMS parameters; its UPD_SLICES slices of lanes sum the
// partials w = slice, slice + UPD_SLICES, ... and the slices are then added
// in slice order (a fixed order: the result is reproducible).
constexpr int UPD_PARAMS = 32;
constexpr int UPD_SLICES = TB / UPD_PARAMS;
constexpr int UPD_GRID = (NPARAM + UPD_PARAMS - 1) / UPD_PARAMS;

__global__ __launch_bounds__(TB) void k_mlp_update(float* __restrict__ params, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ partials,
                                                   int nwg, int mode, float lr, float bc1, float bc2,
                                                   float* __restrict__ grad, const double* __restrict__ lossp,
                                                   double* __restrict__ loss_epoch, int epoch,
                                                   uint16_t* __restrict__ W1b, uint16_t* __restrict__ W2b,
                                                   uint16_t* __restrict__ W3b, uint16_t* __restrict__ W2t,
                                                   uint16_t* __restrict__ W3t, uint16_t* __restrict__ W2p,
                                                   uint16_t* __restrict__ W3p)
{
    __shared__ float part[UPD_SLICES][UPD_PARAMS];
    const int lp = threadIdx.x % UPD_PARAMS, slice = threadIdx.x / UPD_PARAMS;
    const int i = blockIdx.x * UPD_PARAMS + lp;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss_epoch) {
        double s = 0.0;
        for (int w = 0; w < nwg; ++w) s += lossp[w];
        loss_epoch[2 * epoch] += s;
        loss_epoch[2 * epoch + 1] += 1.0;
    }
    float g = 0.f;
    if (i < NPARAM) {
#pragma unroll 8
        for (int w = slice; w < nwg; w += UPD_SLICES) g += partials[(int64_t)w * NPARAM_PAD + i];
    }
    part[slice][lp] = g;
    __syncthreads();
    if (slice != 0 || i >= NPARAM) return;
#pragma unroll
    for (int k = 1; k < UPD_SLICES; ++k) g += part[k][lp];
    if (mode == 1) {
        grad[i] = g;
        return;
    }
    constexpr float B1 = 0.9f, B2 = 0.999f, EPS = 1e-8f;
    const float mi = B1 * m[i] + (1.0f - B1) * g;
    const float vi = B2 * v[i] + (1.0f - B2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float p = params[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + EPS);
    params[i] = p;
    const uint16_t b = bf16_bits(p);
    if (i < OFF_B1) {
        const int h = i / Q, f = i % Q;
        W1b[h * KIN + f] = b;
    } else if (i >= OFF_W2 && i < OFF_B2) {
        const int j = i - OFF_W2, h2 = j / HID, h1 = j % HID;
        W2b[h2 * HID + h1] = b;
        W2t[h1 * HID + h2] = b;
        W2p[h2 * HID + chain_slot(h1)] = f16_bits(p);
    } else if (i >= OFF_W3 && i < OFF_B3) {
        const int j = i - OFF_W3, o = j / HID, h = j % HID;
        W3b[o * HID + h] = b;
        W3t[h * KIN + o] = b;
        W3p[o * HID + chain_slot(h)] = f16_bits(p);
    }
}

// The binary16 GELU of the inference form on x[0..n): eight values per lane,
// through the same packed instructions as the hidden layers.
__global__ __launch_bounds__(TB) void k_gelu16(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, int64_t n)
{
    const int64_t i = 8 * ((int64_t)blockIdx.x * TB + threadIdx.x);
    if (i >= n) return;
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = i + j < n ? (float)__builtin_bit_cast(_Float16, x[i + j]) : 0.0f;
    uint32_t r[4];
    gelu_h2x4(v, r);
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (i + j < n) y[i + j] = (uint16_t)(r[j >> 1] >> (16 * (j & 1)));
}

// Learned equilibrium of n shifted-population sites (one per lane), with the
// plain equilibrium where the verdict is fallback.
template <bool FP8>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_eval(const float* __restrict__ pre, int64_t n, Net net, float threshold,
                                                 float* __restrict__ geq, float* __restrict__ res,
                                                 int32_t* __restrict__ fb)
{
    __shared__ uint16_t lds[TB / 64][WAVE_LDS_BYTES / 2];
    uint16_t* X = lds[threadIdx.x >> 6];
    const int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x;
    const bool active = s < n;
    {
        float in[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) in[p] = active ? pre[s * Q + p] : 0.0f;
        stage_inputs(X, net, in);
    }
    network_outputs<FP8, false>(net, X);
    float g[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) g[p] = active ? pre[s * Q + p] : 0.0f;
    float gh[Q];
    const Verdict vd = learned_equilibrium(g, net, X, threshold, gh);
    if (!active) return;
    if (vd.fallback) {
        const Macro<float> m = macro_from_raw<float, true>(raw_moments_compensated(g));
        relax_emit<float, true>(g, m, 1.0f, 0.0f, [&](int p, float v) { geq[s * Q + p] = v; });
    } else {
#pragma unroll
        for (int p = 0; p < Q; ++p) geq[s * Q + p] = gh[p];
    }
    if (res) res[s] = vd.residual;
    if (fb) fb[s] = vd.fallback ? 1 : 0;
}

// ---- host side ----------------------------------------------------------------------

thread_local char g_mlp_err[512];

int mfail(lb_mlp* m, int code, const char* fmt, ...)
{
    char* dst = m ? m->err : g_mlp_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

int mcheck(lb_mlp* m, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return LB_OK;
    return mfail(m, LB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int fold_norm(lb_mlp* m)
{
    hipLaunchKernelGGL(k_mlp_fold_norm, dim3(1), dim3(64), 0, m->stream, (const float*)m->norm, m->fnorm);
    return mcheck(m, "folding the standardisation");
}

struct WsLayout {
    size_t params, m, v, W1b, W2b, W3b, W2t, W3t, W2p, W3p, W1s, W2q, W3s, b1s, b2s, gk2, norm, fnorm, partials, lossp,
        loss_epoch, stats, grad, total;
};

WsLayout workspace_layout(int max_batch)
{
    const int max_wg = max_batch / TS;
    WsLayout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    l.params = take(NPARAM_PAD * 4);
    l.m = take(NPARAM_PAD * 4);
    l.v = take(NPARAM_PAD * 4);
    l.W1b = take(HID * KIN * 2);
    l.W2b = take(HID * HID * 2);
    l.W3b = take(NOUT * HID * 2);
    l.W2t = take(HID * HID * 2);
    l.W3t = take(HID * KIN * 2);
    l.W2p = take(HID * HID * 2);
    l.W3p = take(NOUT * HID * 2);
    l.W1s = take(HID * KIN * 2);
    l.W2q = take(HID * HID);
    l.W3s = take(NOUT * HID * 2);
    l.b1s = take(HID * 4);
    l.b2s = take(HID * 4);
    l.gk2 = take(16 * 4);
    l.norm = take(4 * 64 * 4);
    l.fnorm = take(4 * 64 * 4);
    l.partials = take((size_t)max_wg * NPARAM_PAD * 4);
    l.lossp = take((size_t)max_wg * 8);
    l.loss_epoch = take((size_t)MAX_EPOCHS * 2 * 8);
    l.stats = take(((size_t)STAT_BLOCKS + 1) * NSTAT * 8);
    l.grad = take(NPARAM_PAD * 4);
    l.total = o;
    return l;
}

int launch_pack_fp8(lb_mlp* m)
{
    hipLaunchKernelGGL(k_mlp_pack_fp8, dim3(1), dim3(TB), 0, m->stream, m->params, m->W1s, m->W2q, m->W3s, m->b1s,
                       m->b2s, m->gk2);
    return mcheck(m, "FP8 pack");
}

// Operand copies of the parameters: the BF16 ones, and the FP8 form's when
// the network evaluates in it.
int launch_pack(lb_mlp* m)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3((HID * HID + TB - 1) / TB), dim3(TB), 0, m->stream, m->params, m->W1b, m->W2b,
                       m->W3b, m->W2t, m->W3t, m->W2p, m->W3p);
    const int rc = mcheck(m, "pack");
    if (rc != LB_OK || m->precision != LB_MLP_FP8) return rc;
    return launch_pack_fp8(m);
}

int reset_adam(lb_mlp* m)
{
    m->adam_t = 0;
    if (hipMemsetAsync(m->adam_m, 0, NPARAM_PAD * 4, m->stream) != hipSuccess ||
        hipMemsetAsync(m->adam_v, 0, NPARAM_PAD * 4, m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "reset of the optimiser state failed");
    return LB_OK;
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Host Philox for the per-epoch order (same generator as the device one).
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1, n3 = (uint32_t)p0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Epoch order i -> (a i + c) mod n: (a, c) from Philox counter (epoch, 0,
// 0xFFFFFFFE, 0); a moved up to the next value coprime with n (wrapping to 1).
void epoch_order(int64_t n, uint64_t seed, int epoch, int64_t& a, int64_t& c)
{
    uint32_t ctr[4] = {(uint32_t)epoch, 0u, 0xFFFFFFFEu, 0u};
    philox_host(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint64_t aa = (uint64_t)ctr[0] % (uint64_t)n;
    if (aa == 0) aa = 1;
    while (gcd64(aa, (uint64_t)n) != 1) aa = aa + 1 < (uint64_t)n ? aa + 1 : 1;
    a = (int64_t)aa;
    c = (int64_t)((uint64_t)ctr[1] % (uint64_t)n);
}

int fwdbwd(lb_mlp* m, const float* pre, const float* post, int64_t n, int64_t a, int64_t c, int64_t start,
           int32_t batch, float tau)
{
    const int nwg = batch / TS;
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(nwg), dim3(TB), 0, m->stream, pre, post, n, a, c, start, (int64_t)batch, tau,
                       m->net(), m->partials, m->lossp);
    return mcheck(m, "forward/backward");
}

}  // namespace

extern "C" {

size_t lb_mlp_workspace_bytes(int32_t max_batch)
{
    if (max_batch < TS || max_batch % TS != 0) return 0;
    return workspace_layout(max_batch).total;
}

size_t lb_mlp_param_count(void) { return NPARAM; }

int lb_mlp_create(lb_mlp** out, void* workspace, size_t bytes, int32_t max_batch, void* stream)
{
    if (!out) return mfail(nullptr, LB_EINVAL, "lb_mlp_create: out is NULL");
    *out = nullptr;
    const size_t need = lb_mlp_workspace_bytes(max_batch);
    if (need == 0) return mfail(nullptr, LB_EINVAL, "lb_mlp_create: max_batch %d must be a positive multiple of %d", max_batch, TS);
    if (!workspace || ((uintptr_t)workspace & 255u)) return mfail(nullptr, LB_EINVAL, "lb_mlp_create: workspace NULL or not 256-byte aligned");
    if (bytes < need) return mfail(nullptr, LB_EINVAL, "lb_mlp_create: workspace %zu < %zu bytes", bytes, need);
    lb_mlp* m = new (std::nothrow) lb_mlp();
    if (!m) return mfail(nullptr, LB_EINVAL, "lb_mlp_create: out of host memory");
    const WsLayout l = workspace_layout(max_batch);
    char* ws = (char*)workspace;
    m->stream = (hipStream_t)stream;
    m->ws = ws;
    m->bytes = bytes;
    m->max_batch = max_batch;
    m->max_wg = max_batch / TS;
    m->params = (float*)(ws + l.params);
    m->adam_m = (float*)(ws + l.m);
    m->adam_v = (float*)(ws + l.v);
    m->W1b = (uint16_t*)(ws + l.W1b);
    m->W2b = (uint16_t*)(ws + l.W2b);
    m->W3b = (uint16_t*)(ws + l.W3b);
    m->W2t = (uint16_t*)(ws + l.W2t);
    m->W3t = (uint16_t*)(ws + l.W3t);
    m->W2p = (uint16_t*)(ws + l.W2p);
    m->W3p = (uint16_t*)(ws + l.W3p);
    m->W1s = (uint16_t*)(ws + l.W1s);
    m->W2q = (uint8_t*)(ws + l.W2q);
    m->W3s = (uint16_t*)(ws + l.W3s);
    m->b1s = (float*)(ws + l.b1s);
    m->b2s = (float*)(ws + l.b2s);
    m->gk2 = (float*)(ws + l.gk2);
    m->precision = LB_MLP_F16;
    m->norm = (float*)(ws + l.norm);
    m->fnorm = (float*)(ws + l.fnorm);
    m->partials = (float*)(ws + l.partials);
    m->lossp = (double*)(ws + l.lossp);
    m->loss_epoch = (double*)(ws + l.loss_epoch);
    m->stats = (double*)(ws + l.stats);
    m->grad = (float*)(ws + l.grad);
    m->adam_t = 0;
    m->err[0] = 0;
    // identity standardisation until one is set or fitted
    float norm[256];
    for (int j = 0; j < 64; ++j) {
        norm[j] = 0.f;
        norm[64 + j] = 1.f;
        norm[128 + j] = 0.f;
        norm[192 + j] = 1.f;
    }
    if (hipMemcpyAsync(m->norm, norm, sizeof norm, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
        hipMemsetAsync(m->params, 0, NPARAM_PAD * 4, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess) {
        snprintf(g_mlp_err, sizeof g_mlp_err, "lb_mlp_create: device initialisation failed");
        delete m;
        return LB_EDEVICE;
    }
    int rc = reset_adam(m);
    if (rc == LB_OK) rc = launch_pack(m);
    if (rc == LB_OK) rc = fold_norm(m);
    if (rc != LB_OK) {
        snprintf(g_mlp_err, sizeof g_mlp_err, "%s", m->err);
        delete m;
        return rc;
    }
    *out = m;
    return LB_OK;
}

void lb_mlp_destroy(lb_mlp* m) { delete m; }

const char* lb_mlp_last_error(const lb_mlp* m) { return m ? m->err : g_mlp_err; }

int lb_mlp_init(lb_mlp* m, uint64_t seed)
{
    if (!m) return mfail(nullptr, LB_EINVAL, "lb_mlp_init: NULL network");
    hipLaunchKernelGGL(k_mlp_init, dim3((NPARAM + TB - 1) / TB), dim3(TB), 0, m->stream, m->params, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    int rc = mcheck(m, "lb_mlp_init");
    if (rc == LB_OK) rc = reset_adam(m);
    if (rc == LB_OK) rc = launch_pack(m);
    return rc;
}

int lb_mlp_set_params(lb_mlp* m, const float* host_params)
{
    if (!m || !host_params) return mfail(m, LB_EINVAL, "lb_mlp_set_params: NULL argument");
    if (hipMemcpyAsync(m->params, host_params, NPARAM * 4, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "lb_mlp_set_params: copy failed");
    int rc = reset_adam(m);
    if (rc == LB_OK) rc = launch_pack(m);
    return rc;
}

int lb_mlp_get_params(lb_mlp* m, float* host_params)
{
    if (!m || !host_params) return mfail(m, LB_EINVAL, "lb_mlp_get_params: NULL argument");
    if (hipMemcpyAsync(host_params, m->params, NPARAM * 4, hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "lb_mlp_get_params: copy failed");
    return LB_OK;
}

int lb_mlp_set_normalization(lb_mlp* m, const float* host_norm)
{
    if (!m || !host_norm) return mfail(m, LB_EINVAL, "lb_mlp_set_normalization: NULL argument");
    float norm[256];
    for (int j = 0; j < 64; ++j) {
        const bool in = j < Q;
        norm[j] = in ? host_norm[j] : 0.f;
        norm[64 + j] = in ? 1.0f / host_norm[Q + j] : 1.f;
        norm[128 + j] = in ? host_norm[2 * Q + j] : 0.f;
        norm[192 + j] = in ? host_norm[3 * Q + j] : 1.f;
    }
    for (int j = 0; j < Q; ++j)
        if (!(host_norm[Q + j] > 0.f) || !(host_norm[3 * Q + j] > 0.f))
            return mfail(m, LB_EINVAL, "lb_mlp_set_normalization: standard deviations must be > 0");
    if (hipMemcpyAsync(m->norm, norm, sizeof norm, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "lb_mlp_set_normalization: copy failed");
    return fold_norm(m);
}

int lb_mlp_get_normalization(lb_mlp* m, float* host_norm)
{
    if (!m || !host_norm) return mfail(m, LB_EINVAL, "lb_mlp_get_normalization: NULL argument");
    float norm[256];
    if (hipMemcpyAsync(norm, m->norm, sizeof norm, hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "lb_mlp_get_normalization: copy failed");
    for (int j = 0; j < Q; ++j) {
        host_norm[j] = norm[j];
        host_norm[Q + j] = 1.0f / norm[64 + j];
        host_norm[2 * Q + j] = norm[128 + j];
        host_norm[3 * Q + j] = norm[192 + j];
    }
    return LB_OK;
}

int lb_mlp_fit_normalization(lb_mlp* m, const float* pre, const float* post, int64_t n, double tau)
{
    if (!m || !pre || !post || n < 1 || !(tau > 0.5)) return mfail(m, LB_EINVAL, "lb_mlp_fit_normalization: bad argument");
    double* partials = m->stats;
    double* mean = m->stats + (size_t)STAT_BLOCKS * NSTAT;
    const int nb = (int)std::min<int64_t>(STAT_BLOCKS, (n + STAT_TILE - 1) / STAT_TILE);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_mlp_stats, dim3(nb), dim3(TB), 0, m->stream, pre, post, n, (float)tau, pass,
                           (const double*)mean, partials);
        hipLaunchKernelGGL(k_mlp_stats_final, dim3(1), dim3(128), 0, m->stream, (const double*)partials, nb, n, pass,
                           mean, m->norm);
    }
    const int rc = mcheck(m, "lb_mlp_fit_normalization");
    return rc == LB_OK ? fold_norm(m) : rc;
}

int lb_mlp_gradient(lb_mlp* m, const float* pre, const float* post, int32_t n, double tau, float* host_grad,
                    double* host_loss)
{
    if (!m || !pre || !post || !host_grad) return mfail(m, LB_EINVAL, "lb_mlp_gradient: NULL argument");
    if (n < TS || n % TS != 0 || n > m->max_batch)
        return mfail(m, LB_EINVAL, "lb_mlp_gradient: n = %d must be a multiple of %d and <= %d", n, TS, m->max_batch);
    int rc = fwdbwd(m, pre, post, n, 1, 0, 0, n, (float)tau);
    if (rc != LB_OK) return rc;
    hipLaunchKernelGGL(k_mlp_update, dim3(UPD_GRID), dim3(TB), 0, m->stream, m->params, m->adam_m,
                       m->adam_v, (const float*)m->partials, n / TS, 1, 0.f, 1.f, 1.f, m->grad,
                       (const double*)m->lossp, (double*)nullptr, 0, m->W1b, m->W2b, m->W3b, m->W2t, m->W3t,
                       m->W2p, m->W3p);
    rc = mcheck(m, "lb_mlp_gradient");
    if (rc != LB_OK) return rc;
    double lossp[4096];
    const int nwg = n / TS;
    if (hipMemcpyAsync(host_grad, m->grad, NPARAM * 4, hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        (host_loss && nwg <= 4096 &&
         hipMemcpyAsync(lossp, m->lossp, nwg * 8, hipMemcpyDeviceToHost, m->stream) != hipSuccess) ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "lb_mlp_gradient: copy failed");
    if (host_loss) {
        double s = 0.0;
        for (int w = 0; w < nwg && w < 4096; ++w) s += lossp[w];
        *host_loss = s;
    }
    return LB_OK;
}

int lb_mlp_train(lb_mlp* m, const float* pre, const float* post, int64_t n, double tau, int32_t batch,
                 int32_t epochs, float lr, uint64_t seed, int64_t max_steps, double* host_epoch_loss)
{
    if (!m || !pre || !post) return mfail(m, LB_EINVAL, "lb_mlp_train: NULL argument");
    if (batch < TS || batch % TS != 0 || batch > m->max_batch)
        return mfail(m, LB_EINVAL, "lb_mlp_train: batch %d must be a multiple of %d and <= %d", batch, TS, m->max_batch);
    if (n < batch) return mfail(m, LB_EINVAL, "lb_mlp_train: %lld pairs < batch %d", (long long)n, batch);
    if (epochs < 1 || epochs > MAX_EPOCHS || !(lr > 0.f) || !(tau > 0.5))
        return mfail(m, LB_EINVAL, "lb_mlp_train: bad epochs, lr or tau");
    if (hipMemsetAsync(m->loss_epoch, 0, (size_t)epochs * 2 * 8, m->stream) != hipSuccess)
        return mfail(m, LB_EDEVICE, "lb_mlp_train: reset of loss history failed");
    const int64_t spe = n / batch;
    const int64_t total = spe * epochs;
    int64_t step = 0;
    for (int e = 0; e < epochs; ++e) {
        int64_t a, c;
        epoch_order(n, seed, e, a, c);
        for (int64_t b = 0; b < spe; ++b) {
            if (max_steps > 0 && step >= max_steps) break;
            int rc = fwdbwd(m, pre, post, n, a, c, b * batch, batch, (float)tau);
            if (rc != LB_OK) return rc;
            const double lr_t = (double)lr * 0.5 * (1.0 + cos(M_PI * (double)step / (double)total));
            m->adam_t += 1;
            const double bc1 = 1.0 - pow(0.9, (double)m->adam_t), bc2 = 1.0 - pow(0.999, (double)m->adam_t);
            hipLaunchKernelGGL(k_mlp_update, dim3(UPD_GRID), dim3(TB), 0, m->stream, m->params,
                               m->adam_m, m->adam_v, (const float*)m->partials, batch / TS, 0, (float)lr_t,
                               (float)bc1, (float)bc2, m->grad, (const double*)m->lossp, m->loss_epoch, e, m->W1b,
                               m->W2b, m->W3b, m->W2t, m->W3t, m->W2p, m->W3p);
            rc = mcheck(m, "lb_mlp_train: update");
            if (rc != LB_OK) return rc;
            ++step;
        }
    }
    // the updates refresh the BF16 copies; the FP8 form's are made once at the end
    if (m->precision == LB_MLP_FP8) {
        const int rc = launch_pack_fp8(m);
        if (rc != LB_OK) return rc;
    }
    if (host_epoch_loss) {
        double* hl = new (std::nothrow) double[(size_t)epochs * 2];
        if (!hl) return mfail(m, LB_EINVAL, "lb_mlp_train: out of host memory");
        const bool ok = hipMemcpyAsync(hl, m->loss_epoch, (size_t)epochs * 16, hipMemcpyDeviceToHost, m->stream) == hipSuccess &&
                        hipStreamSynchronize(m->stream) == hipSuccess;
        if (ok)
            for (int e = 0; e < epochs; ++e) host_epoch_loss[e] = hl[2 * e + 1] > 0 ? hl[2 * e] / hl[2 * e + 1] : NAN;
        delete[] hl;
        if (!ok) return mfail(m, LB_EDEVICE, "lb_mlp_train: copy of the loss history failed");
    }
    return LB_OK;
}

int lb_mlp_equilibrium(lb_mlp* m, const float* pre, int64_t n, float threshold, float* geq, float* residual,
                       int32_t* fallback)
{
    if (!m || !pre || !geq || n < 0) return mfail(m, LB_EINVAL, "lb_mlp_equilibrium: bad argument");
    if (n == 0) return LB_OK;
    if (m->precision == LB_MLP_FP8)
        hipLaunchKernelGGL(k_mlp_eval<true>, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, m->stream, pre, n,
                           m->net(), threshold, geq, residual, fallback);
    else
        hipLaunchKernelGGL(k_mlp_eval<false>, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, m->stream, pre, n,
                           m->net(), threshold, geq, residual, fallback);
    return mcheck(m, "lb_mlp_equilibrium");
}

int lb_mlp_set_precision(lb_mlp* m, int32_t precision)
{
    if (!m) return mfail(nullptr, LB_EINVAL, "lb_mlp_set_precision: NULL network");
    if (precision != LB_MLP_F16 && precision != LB_MLP_FP8)
        return mfail(m, LB_EINVAL, "lb_mlp_set_precision: unknown precision %d", precision);
    m->precision = precision;
    return precision == LB_MLP_FP8 ? launch_pack_fp8(m) : LB_OK;
}

int lb_mlp_get_precision(const lb_mlp* m) { return m ? m->precision : LB_EINVAL; }

int lb_mlp_gelu16(const uint16_t* x, uint16_t* y, int64_t n, void* stream)
{
    if (!x || !y || n < 0) return mfail(nullptr, LB_EINVAL, "lb_mlp_gelu16: bad argument");
    if (n == 0) return LB_OK;
    const int64_t lanes = (n + 7) / 8;  // eight values per lane
    if (lanes > (int64_t)TB * 0x7fffffff) return mfail(nullptr, LB_EINVAL, "lb_mlp_gelu16: n is too large");
    hipLaunchKernelGGL(k_gelu16, dim3((unsigned)((lanes + TB - 1) / TB)), dim3(TB), 0, (hipStream_t)stream, x, y, n);
    return mcheck(nullptr, "lb_mlp_gelu16");
}

int lb_pairgen(float* pre, float* post, int64_t n, uint64_t seed, double tau, void* stream)
{
    if (!pre || !post || n < 0 || !(tau > 0.5)) return mfail(nullptr, LB_EINVAL, "lb_pairgen: bad argument");
    if (n == 0) return LB_OK;
    hipLaunchKernelGGL(k_pairgen, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, (hipStream_t)stream, pre, post, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), (float)(1.0 / tau));
    return mcheck(nullptr, "lb_pairgen");
}

}  // extern "C"
