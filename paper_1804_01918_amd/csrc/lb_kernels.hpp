// HIP kernels of the D2Q37 step: init, propagate, collide, the fused step,
// FP64 readouts (moments, canonical populations) and the FP64 audit.
#pragma once

#include "lb_collide.hpp"

namespace d2q37 {

constexpr int BLOCK = 256;

// ---- FP64 conversions of stored values ------------------------------------

// Stored value -> FP64 f (plain) or g (shifted). Exact for every precision.
template <class P>
__device__ inline double load_f64(const typename P::T* a, int p)
{
    if constexpr (P::kind == PREC_F16S)
        return (double)__half2float(__ushort_as_half(*a)) / (double)S16[shell_of_c2(c2_of(p))];
    else
        return (double)*a;
}

// Round an FP64 value to nearest-even FP16 without double rounding: first to
// FP32 with round-to-odd (truncate, then set the last bit if inexact), which
// keeps enough bits for the final FP32 -> FP16 rounding to be correct.
__device__ inline uint16_t f64_to_f16_rne(double x)
{
    float f = __double2float_rz(x);
    if ((double)f != x && x == x) {
        uint32_t b = __float_as_uint(f);
        b |= 1u;
        f = __uint_as_float(b);
    }
    return __half_as_ushort(__float2half_rn(f));
}

// FP64 f (plain) or g (shifted) -> stored value, rounding to nearest even.
template <class P>
__device__ inline void store_from_f64(typename P::T* a, int p, double v)
{
    if constexpr (P::kind == PREC_F16S)
        *a = f64_to_f16_rne(v * (double)S16[shell_of_c2(c2_of(p))]);
    else
        *a = (typename P::T)v;
}

// The compute value as it will read back after storage (FP16 rounds).
template <class P>
__device__ inline double stored_as_f64(typename P::C v, int p)
{
    if constexpr (P::kind == PREC_F16S) {
        const float s = S16[shell_of_c2(c2_of(p))];
        return (double)__half2float(__float2half_rn(v * s)) / (double)s;
    } else {
        return (double)v;
    }
}

// ---- FP64 audit ------------------------------------------------------------
// Per site: {sum v, R sum cx v, R sum cy v, R^2/2 sum |c|^2 v}, i.e. mass,
// momentum and energy (1/2 sum f xi^2) of f, or of g for shifted storage
// (the constant part 1, 0, 0, 1 per site is added at finalisation).
__device__ inline void audit_site(const double (&d)[Q], double (&acc)[4])
{
    double m = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        m += d[p];
        if (CX[p] != 0) jx += (double)CX[p] * d[p];
        if (CY[p] != 0) jy += (double)CY[p] * d[p];
        if (c2_of(p) != 0) e += (double)c2_of(p) * d[p];
    }
    acc[0] += m;
    acc[1] += R * jx;
    acc[2] += R * jy;
    acc[3] += 0.5 * R2 * e;
}

// Fixed-tree block reduction of 4 doubles (wavefront butterfly, then the 4
// wavefronts of the block in order); thread 0 writes out[0..3].
__device__ inline void block_reduce4(double (&acc)[4], double* out)
{
    __shared__ double red[BLOCK / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[wave][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double s = red[0][k];
            for (int w = 1; w < BLOCK / 64; ++w) s += red[w][k];
            out[k] = s;
        }
    }
}

// ---- walls ------------------------------------------------------------------
// Diffuse walls at rest on the planes y = -1/2 (wall 0, bottom) and
// y = LY - 1/2 (wall 1, top), each at its own temperature; x stays periodic.
// In the pull propagate a population whose source row lies beyond a wall is
// emitted by that wall: the equilibrium at rest and the wall's temperature,
// with the density rho_w of its source column fixed so that the wall emits
// from each column exactly the mass that left the fluid towards it from
// that column in the same propagate (Ansumali and Karlin's diffuse
// reflection, written for a lattice whose hops reach three rows).
//
// No extra rows are stored: a periodic pull that crosses a wall reads a
// slot holding a population that leaves through the opposite wall (for
// c_y > 0 the rows LY - c_y .. LY - 1, for c_y < 0 the rows 0 .. -c_y - 1),
// and that slot has no other reader. k_wall therefore, per column x, sums
// those leaving values into the two wall densities and then overwrites each
// of them with the emission its one reader needs: the bottom wall's for the
// slots that leave through the top, and the other way round. The unchanged
// periodic kernels then pull the walls' emission. (The current buffer is
// changed only in these dead slots, just before it is propagated.)
//
// Wall table (FP64, per wall, WALL_TAB values), made once by k_wall_setup:
//   [0, Q)    A_p = f_eq_p(1, 0, T_w)
//   [Q, 2Q)   B_p = A_p - w_p, from the shifted equilibrium (no cancellation)
//   [2Q]      K  = sum over the populations leaving the wall of |c_y| A_p
//   [2Q + 1]  D  = the same sum of |c_y| B_p (K minus its value at T_w = 1)
//   [2Q + 2]  K and [2Q + 3] D again, from A_p and B_p rounded to FP32: the
//             shifted kernels emit with FP32 A_p, B_p, and with these sums
//             the emitted mass equals the outgoing mass up to FP32
//             arithmetic rounding, with no bias from the rounded constants.
constexpr int WALL_TAB = 2 * Q + 4;

__global__ void k_wall_setup(double* __restrict__ tab, double t_bottom, double t_top)
{
    const int wall = threadIdx.x;
    if (wall >= 2) return;
    double* t = tab + wall * WALL_TAB;
    const double T = wall == 0 ? t_bottom : t_top;
    equilibrium_f64<false>(1.0, 0.0, 0.0, T, [&](int p, double v) { t[p] = v; });
    equilibrium_f64<true>(1.0, 0.0, 0.0, T, [&](int p, double v) { t[Q + p] = v; });
    double k = 0.0, d = 0.0, k32 = 0.0, d32 = 0.0;
    for (int p = 0; p < Q; ++p) {
        const int cy = CY[p];
        if (wall == 0 ? cy > 0 : cy < 0) {
            const double n = (double)(cy > 0 ? cy : -cy);
            k += n * t[p];
            d += n * t[Q + p];
            k32 += n * (double)(float)t[p];
            d32 += n * (double)(float)t[Q + p];
        }
    }
    t[2 * Q] = k;
    t[2 * Q + 1] = d;
    t[2 * Q + 2] = k32;
    t[2 * Q + 3] = d32;
}

// The slots that leave the fluid towards a wall in one propagate: for the
// bottom wall the populations with c_y < 0 in rows j < -c_y, for the top one
// those with c_y > 0 in rows LY - 1 - j, j < c_y; 26 per wall and column,
// listed as (p, j) with the FP16 storage scale of p and its inverse.
struct WallPairs {
    int8_t p[2][32];
    int8_t j[2][32];
    float s16[2][32];
    float inv_s16[2][32];
};
constexpr WallPairs make_wall_pairs()
{
    WallPairs w{};
    for (int wall = 0; wall < 2; ++wall) {
        int k = 0;
        for (int p = 0; p < Q; ++p) {
            const int cy = CY[p];
            if (cy == 0 || (wall == 0) != (cy < 0)) continue;
            const int n = cy > 0 ? cy : -cy;
            for (int j = 0; j < n; ++j) {
                w.p[wall][k] = (int8_t)p;
                w.j[wall][k] = (int8_t)j;
                w.s16[wall][k] = S16[shell_of_c2(c2_of(p))];
                w.inv_s16[wall][k] = 1.0f / S16[shell_of_c2(c2_of(p))];
                ++k;
            }
        }
        for (; k < 32; ++k) {
            w.p[wall][k] = -1;
            w.j[wall][k] = 0;
            w.s16[wall][k] = 0.0f;
            w.inv_s16[wall][k] = 0.0f;
        }
    }
    return w;
}
static __constant__ WallPairs WALL_PAIRS = make_wall_pairs();

// One wavefront per column x of the current buffer: lanes 0..25 hold the
// slots leaving towards the bottom wall, lanes 32..57 those leaving towards
// the top one. Each half is summed in a fixed butterfly order into its
// wall's density; then every slot receives the other wall's emission for
// its population (see the comment above).
template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_wall(typename P::T* __restrict__ buf, Geo g,
                                                const double* __restrict__ tab)
{
    using C = typename P::C;
    constexpr int VL = vl_of<P>();
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    if (col >= g.lx) return;  // whole wavefronts
    const int x = (int)col;
    const int wall = lane >> 5, k = lane & 31;
    const int p = WALL_PAIRS.p[wall][k];
    typename P::T* a = nullptr;
    C v = C(0);
    if (p >= 0) {
        const int j = WALL_PAIRS.j[wall][k];
        const int y = wall == 0 ? j : g.ly - 1 - j;
        if (y >= 0 && y < g.ly) {
            a = const_cast<typename P::T*>(site_ptr<L, VL>((const typename P::T*)buf, x, y, p, g));
            if constexpr (P::kind == PREC_F16S)
                v = __half2float(__ushort_as_half(*a)) * WALL_PAIRS.inv_s16[wall][k];
            else
                v = *a;
        }
    }
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    // v: this half's outgoing mass; the other half's is 32 lanes away
    const C other = __shfl_xor(v, 32, 64);
    if (a) {
        // the slot leaves through `wall`; its reader pulls through the other one
        const int ew = 1 - wall;
        const double* w = tab + ew * WALL_TAB;
        C e;
        if constexpr (P::shifted) {
            const C rw1 = (other - (C)w[2 * Q + 3]) / (C)w[2 * Q + 2];  // rho_w - 1
            e = fma_(rw1, (C)w[p], (C)w[Q + p]);
        } else {
            e = (other / (C)w[2 * Q]) * w[p];
        }
        if constexpr (P::kind == PREC_F16S)
            *a = (uint16_t)__half_as_ushort(__float2half_rn(e * WALL_PAIRS.s16[wall][k]));
        else
            *a = e;
    }
}

// ---- kernels ---------------------------------------------------------------
// Every lattice kernel is launched row-tiled: LX * tpr workgroups of BLOCK
// lanes (see row_tile_site).

#define D2Q37_SITE(P, L)                                        \
    using Elem = typename P::T;                                 \
    constexpr int VL = vl_of<P>();                              \
    int xrow, r;                                                \
    int64_t tile;                                               \
    const bool active = row_tile_site<BLOCK>(g, xrow, r, tile); \
    Stencil<L, Elem, VL> st;                                    \
    if (active) st.setup(xrow, r, g)

template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_init(typename P::T* __restrict__ dst, Geo g,
                                                const double* __restrict__ rho,
                                                const double* __restrict__ ux,
                                                const double* __restrict__ uy,
                                                const double* __restrict__ T)
{
    D2Q37_SITE(P, L);
    if (!active) return;
    const int64_t site = (int64_t)st.x * g.ly + st.y;
    equilibrium_f64<P::shifted>(rho[site], ux[site], uy[site], T[site],
                                [&](int p, double v) { store_from_f64<P>(st.own(dst, p, g), p, v); });
}

// Pure gather, bit copy of every population from its upstream site.
template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_propagate(const typename P::Word* __restrict__ src,
                                                     typename P::Word* __restrict__ dst, Geo g)
{
    using W = typename P::Word;
    constexpr int VL = vl_of<P>();
    int xrow, r;
    int64_t tile;
    if (!row_tile_site<BLOCK>(g, xrow, r, tile)) return;
    Stencil<L, W, VL> st;
    st.setup(xrow, r, g);
    W w[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) w[p] = ld_stream<W, L::stream_loads>(st.src(src, p, g));
    // 2-byte words are stored without the streaming hint (see PrecF16S::store)
#pragma unroll
    for (int p = 0; p < Q; ++p) st_stream<W, L::stream_stores && (sizeof(W) > 2)>(st.own(dst, p, g), w[p]);
}

// Collide in place on the current buffer (with the body force if FORCE).
template <class P, class L, bool COMP, bool FORCE>
__global__ __launch_bounds__(BLOCK) void k_collide(typename P::T* __restrict__ buf, Geo g, double omega,
                                                   Force<typename P::C> force)
{
    using C = typename P::C;
    D2Q37_SITE(P, L);
    if (!active) return;
    C v[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) v[p] = P::template load<L::stream_loads>(st.own(buf, p, g), p);
    collide_site_f<P, COMP, FORCE>(v, (C)omega, force,
                                   [&](int p, C res) { P::template store<L::stream_stores>(st.own(buf, p, g), p, res); });
}

// Fused step src -> dst: pull the 37 populations, collide, store at the own
// site. With AUDIT, the FP64 mass/momentum/energy of the stored result are
// reduced per workgroup into partials[4 * tile]. With FORCE, the collide
// applies the body force (zero force rounds exactly as without it). Walls
// need nothing here: k_wall has put their emission into the slots the pull
// reads.
template <class P, class L, bool COMP, bool AUDIT, bool FORCE>
__global__ __launch_bounds__(BLOCK) void k_step(const typename P::T* __restrict__ src,
                                                typename P::T* __restrict__ dst, Geo g, double omega,
                                                double* __restrict__ partials, Force<typename P::C> force)
{
    using C = typename P::C;
    D2Q37_SITE(P, L);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        C v[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) v[p] = P::template load<L::stream_loads>(st.src(src, p, g), p);
        if constexpr (AUDIT) {
            double d[Q];
            collide_site_f<P, COMP, FORCE>(v, (C)omega, force, [&](int p, C res) {
                P::template store<L::stream_stores>(st.own(dst, p, g), p, res);
                d[p] = stored_as_f64<P>(res, p);
            });
            audit_site(d, acc);
        } else {
            collide_site_f<P, COMP, FORCE>(v, (C)omega, force, [&](int p, C res) {
                P::template store<L::stream_stores>(st.own(dst, p, g), p, res);
            });
        }
    } else if (!AUDIT) {
        return;
    }
    if constexpr (AUDIT) block_reduce4(acc, partials + 4 * tile);
}

template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_audit(const typename P::T* __restrict__ buf, Geo g,
                                                 double* __restrict__ partials)
{
    D2Q37_SITE(P, L);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        double d[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) d[p] = load_f64<P>(st.own(buf, p, g), p);
        audit_site(d, acc);
    }
    block_reduce4(acc, partials + 4 * tile);
}

// Deterministic final sum of nparts partials (strided per thread, then the
// fixed block tree); adds `base` (the per-site constant of shifted storage
// times the site count).
__global__ __launch_bounds__(BLOCK) void k_audit_final(const double* __restrict__ partials, int64_t nparts,
                                                       double4 base, double* __restrict__ out)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < nparts; i += BLOCK) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += partials[4 * i + k];
    }
    __shared__ double res[4];
    block_reduce4(acc, res);
    if (threadIdx.x == 0) {
        out[0] = base.x + res[0];
        out[1] = base.y + res[1];
        out[2] = base.z + res[2];
        out[3] = base.w + res[3];
    }
}

// FP64 macroscopic fields (thermal units) of the stored state.
template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_moments(const typename P::T* __restrict__ buf, Geo g,
                                                   double* __restrict__ rho, double* __restrict__ ux,
                                                   double* __restrict__ uy, double* __restrict__ T)
{
    D2Q37_SITE(P, L);
    if (!active) return;
    double d[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) d[p] = load_f64<P>(st.own(buf, p, g), p);
    const RawMoments<double> m = raw_moments_plain<double>(d);
    const Macro<double> s = macro_from_raw<double, P::shifted>(m);
    const int64_t site = (int64_t)st.x * g.ly + st.y;
    rho[site] = s.rho;
    ux[site] = s.Ux / R;
    uy[site] = s.Uy / R;
    T[site] = 1.0 + s.t;
}

// Stored state -> canonical FP64 f[p][x][y].
template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_get(const typename P::T* __restrict__ buf, Geo g,
                                               double* __restrict__ f)
{
    D2Q37_SITE(P, L);
    if (!active) return;
    const int64_t site = (int64_t)st.x * g.ly + st.y;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const double d = load_f64<P>(st.own(buf, p, g), p);
        f[(int64_t)p * g.n + site] = P::shifted ? weight(p) + d : d;
    }
}

// Canonical FP64 f[p][x][y] -> stored state.
template <class P, class L>
__global__ __launch_bounds__(BLOCK) void k_set(typename P::T* __restrict__ buf, Geo g,
                                               const double* __restrict__ f)
{
    D2Q37_SITE(P, L);
    if (!active) return;
    const int64_t site = (int64_t)st.x * g.ly + st.y;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const double d = f[(int64_t)p * g.n + site];
        store_from_f64<P>(st.own(buf, p, g), p, P::shifted ? d - weight(p) : d);
    }
}

// Streaming copy of 16-byte words (the achievable-bandwidth reference): one
// word per thread, streaming hints on both sides. Of the forms measured on
// this GPU (1, 2 or 4 words per thread, 256 to 1024 threads per workgroup,
// grid-stride loops, with or without the hints) this one moves the most.
constexpr int COPY_UNROLL = 1;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(BLOCK) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                  int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n16) st_stream(dst + i, ld_stream(src + i));
}

}  // namespace d2q37
