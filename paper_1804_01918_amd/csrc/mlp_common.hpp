// Learned collide: shared device pieces of the MLP 37 -> 128 -> 128 -> 37
// (GELU), run on the gfx950 matrix cores with FP32 accumulation: trained in
// BF16, evaluated with a BF16 first layer and binary16 hidden layers (or an
// FP8 hidden layer).
//
// Matrix-core tiles: v_mfma_f32_16x16x32_bf16 computes D(16x16) += A(16x32)
// B(32x16). Lane l of the wavefront holds
//   A: row l % 16, columns k = 8 (l / 16) + 0..7      (8 bf16)
//   B: column l % 16, rows  k = 8 (l / 16) + 0..7      (8 bf16)
//   D: column l % 16, rows  4 (l / 16) + 0..3          (4 float)
// so both operands are "16 indices x 32 k" fragments: lane l takes index
// l % 16 and eight consecutive k. With a matrix stored index-major (k
// contiguous) a fragment is one 16-byte load per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lb_collide.hpp"

namespace d2q37 {
namespace mlp {

constexpr int HID = 128;
constexpr int KIN = 64;    // input features padded 37 -> 64 (two 32-wide k steps)
constexpr int NOUT = 48;   // outputs padded 37 -> 48 (three 16-wide tiles)
// Packed FP32 parameter vector: W1[128][37], b1[128], W2[128][128], b2[128],
// W3[37][128], b3[37].
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + HID * Q;
constexpr int OFF_W2 = OFF_B1 + HID;
constexpr int OFF_B2 = OFF_W2 + HID * HID;
constexpr int OFF_W3 = OFF_B2 + HID;
constexpr int OFF_B3 = OFF_W3 + Q * HID;
constexpr int NPARAM = OFF_B3 + Q;  // 26149

constexpr float GELU_C = 0.79788456080286535588f;  // sqrt(2 / pi)
constexpr float GELU_A = 0.044715f;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// FP32 -> BF16, round to nearest even (gfx950 converts in hardware,
// v_cvt_pk_bf16_f32, two values per instruction).
__device__ inline __bf16 to_bf16(float f) { return (__bf16)f; }
__device__ inline uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, to_bf16(f)); }
__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// gelu(a) = 0.5 a (1 + tanh(c (a + A a^3))) written as a / (1 + exp(-2 c (a + A a^3))).
__device__ inline float gelu(float a)
{
    const float y = a * __builtin_fmaf(2.0f * GELU_C * GELU_A, a * a, 2.0f * GELU_C);
    return a / (1.0f + __expf(-y));
}
// The same with the hardware base-2 exponential and reciprocal (about 1 ulp
// each) and log2(e) folded into the constants, for activations that are
// rounded to BF16 right after.
constexpr float GELU_K1 = -2.0f * 1.44269504088896340736f * GELU_C * GELU_A;
constexpr float GELU_K2 = -2.0f * 1.44269504088896340736f * GELU_C;
__device__ inline float gelu_fast(float a)
{
    const float y2 = a * __builtin_fmaf(GELU_K1, a * a, GELU_K2);
    return a * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(y2));
}
__device__ inline float gelu_grad(float a)
{
    const float y = a * __builtin_fmaf(2.0f * GELU_C * GELU_A, a * a, 2.0f * GELU_C);
    const float s = 1.0f / (1.0f + __expf(-y));
    const float dy = __builtin_fmaf(6.0f * GELU_C * GELU_A, a * a, 2.0f * GELU_C);
    return __builtin_fmaf(a * s * (1.0f - s), dy, s);
}

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

// Fragment (indices i0..i0+15, k0..k0+31) of a matrix stored index-major:
// element (i, k) at base[i * ld + k]; ld and k0 multiples of 8.
__device__ inline bf16x8 frag_im(const uint16_t* base, int ld, int i0, int k0)
{
    const int l = lane_id();
    return *(const bf16x8*)(base + (i0 + (l & 15)) * ld + k0 + 8 * (l >> 4));
}
// Same fragment of a matrix stored k-major: element (i, k) at base[k * ld + i].
__device__ inline bf16x8 frag_km(const uint16_t* base, int ld, int i0, int k0)
{
    const int l = lane_id();
    const uint16_t* p = base + (k0 + 8 * (l >> 4)) * ld + i0 + (l & 15);
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = __builtin_bit_cast(__bf16, p[j * ld]);
    return v;
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Binary16 (IEEE half) tiles: v_mfma_f32_16x16x32_f16 has the BF16 lane
// layout; the hidden layers of inference run on it (see gelu_h2x2).
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
__device__ inline f32x4 mfma_f16(u32x4v a, u32x4v b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                 0, 0);
}
__host__ __device__ inline uint16_t f16_bits(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }

// GELU of FP32 pre-activations in binary16 arithmetic, two pairs at a time,
// (a, b) into r0 and (c, d) into r1, each pair packed in one word (first
// value low): every operation rounds to nearest even in binary16,
//   x = h(a), y = x (K1 x^2 + K2) (the K1 product and K2 sum fused), e = 2^y,
//   r = 1 / (1 + e), result x r,
// with K1, K2 of gelu_fast rounded to binary16. Packed instructions take
// both halves at once; the hardware exponential and reciprocal of binary16
// are correctly rounded (checked over every binary16 input), so the result
// is a fixed function of the inputs that a host can reproduce bit for bit.
// The half-word results of the transcendentals are written in place (SDWA):
// the second write of a register reads the first one's result, which needs
// one wait state after a partial-register write on this GPU; the writes of
// the two pairs alternate, so each is the other's wait state.
__device__ inline void gelu_h2x2(float a, float b, float c, float d, uint32_t& r0, uint32_t& r1)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f16x2 x0 = __builtin_convertvector((f32x2){a, b}, f16x2);
    const f16x2 x1 = __builtin_convertvector((f32x2){c, d}, f16x2);
    const f16x2 k1 = {(_Float16)GELU_K1, (_Float16)GELU_K1}, k2 = {(_Float16)GELU_K2, (_Float16)GELU_K2};
    const f16x2 y0 = x0 * __builtin_elementwise_fma(k1, x0 * x0, k2);
    const f16x2 y1 = x1 * __builtin_elementwise_fma(k1, x1 * x1, k2);
    uint32_t e0, e1, q0, q1;
    asm("v_exp_f16_sdwa %0, %2 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"
        "v_exp_f16_sdwa %1, %3 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"
        "v_exp_f16_sdwa %0, %2 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1\n\t"
        "v_exp_f16_sdwa %1, %3 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1"
        : "=&v"(e0), "=&v"(e1)
        : "v"(__builtin_bit_cast(uint32_t, y0)), "v"(__builtin_bit_cast(uint32_t, y1)));
    const f16x2 one = {(_Float16)1, (_Float16)1};
    const f16x2 d0 = __builtin_bit_cast(f16x2, e0) + one, d1 = __builtin_bit_cast(f16x2, e1) + one;
    asm("v_rcp_f16_sdwa %0, %2 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"
        "v_rcp_f16_sdwa %1, %3 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"
        "v_rcp_f16_sdwa %0, %2 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1\n\t"
        "v_rcp_f16_sdwa %1, %3 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1"
        : "=&v"(q0), "=&v"(q1)
        : "v"(__builtin_bit_cast(uint32_t, d0)), "v"(__builtin_bit_cast(uint32_t, d1)));
    r0 = __builtin_bit_cast(uint32_t, x0 * __builtin_bit_cast(f16x2, q0));
    r1 = __builtin_bit_cast(uint32_t, x1 * __builtin_bit_cast(f16x2, q1));
}

// gelu_h2x2 of four pairs, v[2i], v[2i + 1] into r[i].
__device__ inline void gelu_h2x4(const float (&v)[8], uint32_t (&r)[4])
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f16x2 k1 = {(_Float16)GELU_K1, (_Float16)GELU_K1}, k2 = {(_Float16)GELU_K2, (_Float16)GELU_K2};
    f16x2 x[4];
    uint32_t y[4], e[4], dd[4], q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = __builtin_convertvector((f32x2){v[2 * i], v[2 * i + 1]}, f16x2);
        y[i] = __builtin_bit_cast(uint32_t, x[i] * __builtin_elementwise_fma(k1, x[i] * x[i], k2));
    }
#define D2Q37_TRANS4(OP, D, S)                                                                  \
    asm(OP " %0, %4 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"             \
        OP " %1, %5 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"             \
        OP " %2, %6 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"             \
        OP " %3, %7 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_0\n\t"             \
        OP " %0, %4 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1\n\t"             \
        OP " %1, %5 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1\n\t"             \
        OP " %2, %6 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1\n\t"             \
        OP " %3, %7 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1"                  \
        : "=&v"(D[0]), "=&v"(D[1]), "=&v"(D[2]), "=&v"(D[3])                                   \
        : "v"(S[0]), "v"(S[1]), "v"(S[2]), "v"(S[3]))
    D2Q37_TRANS4("v_exp_f16_sdwa", e, y);
    const f16x2 one = {(_Float16)1, (_Float16)1};
#pragma unroll
    for (int i = 0; i < 4; ++i) dd[i] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, e[i]) + one);
    D2Q37_TRANS4("v_rcp_f16_sdwa", q, dd);
#undef D2Q37_TRANS4
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = __builtin_bit_cast(uint32_t, x[i] * __builtin_bit_cast(f16x2, q[i]));
}

// FP8 (e4m3, the OCP variant without infinities) tiles:
// v_mfma_f32_16x16x32_fp8_fp8 has the lane layout above with eight one-byte
// values per lane (one 64-bit register pair per operand).
__device__ inline f32x4 mfma_fp8(uint64_t a, uint64_t b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)a, (long)b, c, 0, 0, 0);
}
// Fragment of a byte matrix stored index-major (ld and k0 multiples of 8).
__device__ inline uint64_t frag8_im(const uint8_t* base, int ld, int i0, int k0)
{
    const int l = lane_id();
    return *(const uint64_t*)(base + (i0 + (l & 15)) * ld + k0 + 8 * (l >> 4));
}
// Two FP32 values rounded to e4m3 (nearest even; beyond the largest finite
// value, 448, the result is NaN), into bytes 2 HI, 2 HI + 1 of `old`.
template <bool HI>
__device__ inline uint32_t pack_fp8(float a, float b, uint32_t old)
{
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, (int)old, HI);
}

// FP8 form of the hidden layer (inference only): its inputs, the GELU
// outputs of the first layer, are scaled by FP8_ACT_SCALE and its weights
// W2 by 2^aw (aw: the largest weight lands in [128, 256)), both rounded to
// e4m3; the product's scale 2^(aw + 4) is carried by copies of W1, b1, b2,
// W3 and by the GELU constants, all scaled by powers of two, so that no
// operation is added and every rounding is that of the unscaled form.
constexpr float FP8_ACT_SCALE = 16.0f;

// Register chaining of layers (inference). Computing a layer transposed,
// H^T (hidden x sites) = W x X^T, each lane ends with 4 consecutive hidden
// units of one site per 16-row tile; two tiles (hidden 16 apart) fill the 8
// k-slots of the next layer's B fragment for that site. So the next layer's
// k index runs over hidden units in the order
//   slot 8q + j of a 32-wide k block  <->  hidden 4q + j (j < 4), 16 + 4q + j - 4 (j >= 4),
// and its weight columns are stored permuted the same way.
__host__ __device__ constexpr int chain_hidden(int slot)
{
    return (slot & ~31) + (((slot & 7) < 4) ? 4 * ((slot & 31) >> 3) + (slot & 7)
                                             : 16 + 4 * ((slot & 31) >> 3) + (slot & 7) - 4);
}
__host__ __device__ constexpr int chain_slot(int hidden)
{
    return (hidden & ~31) + 8 * ((hidden & 15) >> 2) + (hidden & 3) + ((hidden & 16) ? 4 : 0);
}

// Device view of a network: BF16 operand copies (training, and the first
// layer of inference), binary16 copies of W2 and W3 (inference), FP32 biases
// (inside the packed parameters) and the standardisation of inputs and
// outputs.
struct Net {
    const uint16_t* W1b;  // [128][64]  W1[h][f], f padded with zeros
    const uint16_t* W2b;  // [128][128] W2[h2][h1]
    const uint16_t* W3b;  // [48][128]  W3[o][h], o padded with zeros
    const uint16_t* W2t;  // [128][128] W2[h2][h1] at [h1][h2]
    const uint16_t* W3t;  // [128][64]  W3[o][h] at [h][o], o padded
    const uint16_t* W2p;  // [128][128] W2[h2][chain_hidden(slot)] at [h2][slot], binary16
    const uint16_t* W3p;  // [48][128]  W3[o][chain_hidden(slot)] at [o][slot], o padded, binary16
    const float* params;  // packed FP32 parameters (biases read from here)
    const float* norm;    // [4][64]: mean z, 1/sd z, mean y, sd y
    const float* fnorm;   // [4][64] folded for inference: 1/(sd_z w), -mean_z/sd_z, w sd_y, w mean_y
    int ld1 = KIN;        // row strides of W1b and of W2p / W3p (the LDS copies are padded)
    int ld23 = HID;
    // FP8 form: W1 x 16 (BF16 [128][64]), W2 x 2^aw (e4m3 [128][128], chained
    // columns as W2p), W3 x 2^-(aw + 4) (BF16 [48][128], as W3p), b1 x 16,
    // b2 x 2^(aw + 4), and the second GELU's constants for inputs scaled by
    // 2^(aw + 4): {K1 2^-3(aw + 4), K2 2^-(aw + 4)}
    const uint16_t* W1s = nullptr;
    const uint8_t* W2q = nullptr;
    const uint16_t* W3s = nullptr;
    const float* b1s = nullptr;
    const float* b2s = nullptr;
    const float* gk2 = nullptr;
    int ldq = HID;        // row stride of W2q in bytes
    // LDS copies of the biases of the form in use (set by share_weights;
    // otherwise they are read from params, or b1s / b2s in the FP8 form)
    const float* lb1 = nullptr;
    const float* lb2 = nullptr;
    const float* lb3 = nullptr;
};

// ---- conserved part and residual of shifted populations -----------------------
// The four conserved functions phi = 1, xi_x, xi_y, xi^2 - 2 have Gram matrix
// sum_p w_p phi_a phi_b = diag(1, 1, 1, 4) on the D2Q37 quadrature, so the
// projection of g onto w * phi (in the 1/w inner product) has coefficients
// (sum g, sum g xi_x, sum g xi_y, sum g (xi^2 - 2) / 4).
struct Conserved {
    float m0, mx, my, mE;
};

__device__ inline Conserved conserved_moments(const float (&g)[Q])
{
    float m0 = 0.f, jx = 0.f, jy = 0.f, e = 0.f;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        m0 += g[p];
        if (CX[p] != 0) jx = __builtin_fmaf((float)CX[p], g[p], jx);
        if (CY[p] != 0) jy = __builtin_fmaf((float)CY[p], g[p], jy);
        if (c2_of(p) != 0) e = __builtin_fmaf((float)c2_of(p), g[p], e);
    }
    Conserved c;
    c.m0 = m0;
    c.mx = mulk(jx, R);
    c.my = mulk(jy, R);
    c.mE = mulk(e, R2) - 2.0f * m0;
    return c;
}

// Coefficients of a conserved-space vector w_p (a0 + ax xi_px + ay xi_py +
// aE (xi_p^2 - 2) / 4), pre-scaled so that each population needs integer
// multiples only: v_p = c0 + cx cx_p + cy cy_p + cq |c_p|^2, times w_p. The
// model constants enter through hi + lo products (mulk), so the moments of
// the vector are exact to FP32 rounding of the sums.
struct ConservedCoef {
    float c0, cx, cy, cq;
};
__device__ inline ConservedCoef conserved_coef(float a0, float ax, float ay, float aE)
{
    ConservedCoef k;
    k.c0 = a0 - 0.5f * aE;
    k.cx = mulk(ax, R);
    k.cy = mulk(ay, R);
    k.cq = mulk(0.25f * aE, R2);
    return k;
}
__device__ inline float conserved_value(int p, const ConservedCoef& k)
{
    float v = k.c0;
    if (CX[p] != 0) v = __builtin_fmaf(k.cx, (float)CX[p], v);
    if (CY[p] != 0) v = __builtin_fmaf(k.cy, (float)CY[p], v);
    if (c2_of(p) != 0) v = __builtin_fmaf(k.cq, (float)c2_of(p), v);
    return mulk(v, weight(p));
}

// ---- features of a training pair --------------------------------------------------
// z = pre / w; y = (g_eq - P(pre)) / w with g_eq = pre + tau (post - pre).
__device__ inline void pair_features(const float* pre_row, const float* post_row, float tau, float (&z)[Q],
                                     float (&y)[Q])
{
    float g[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) g[p] = pre_row[p];
    const Conserved m = conserved_moments(g);
    const ConservedCoef k = conserved_coef(m.m0, m.mx, m.my, m.mE);
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const float inv_w = (float)(1.0 / weight(p));
        const float geq = __builtin_fmaf(tau, post_row[p] - g[p], g[p]);
        z[p] = g[p] * inv_w;
        y[p] = (geq - conserved_value(p, k)) * inv_w;
    }
}

}  // namespace mlp
}  // namespace d2q37
