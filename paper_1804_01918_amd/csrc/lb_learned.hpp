// Lattice kernels of the learned collide (FP32-shifted storage): the fused
// step and the in-place collide with the network's equilibrium, falling back
// per site to the plain FP32 collide; fallback and site counts are
// accumulated in two 64-bit counters.
//
// Persistent launch: one 512-lane workgroup per compute unit copies the
// weights into LDS once and then walks 512-site row tiles (a tile is a run
// of one lattice row; the tiles of an XCD are contiguous). Each wavefront
// stages its 64 sites' inputs in its own LDS rows, runs the network, then
// gathers the populations a second time (cache hits) for the projection,
// the fallback verdict and the relaxation. Sites that fall back are queued
// per wavefront and collided 64 at a time with the plain FP32 collide, so
// that a few fallback lanes do not hold a whole wavefront in it: the site
// index goes to LDS, the site's pulled populations (in registers at that
// point) to the wavefront's slots of a ring in the caller's scratch, so that
// a batch reads 64 compact slots instead of gathering again from 37 lines
// per site.
#pragma once

#include "lb_kernels.hpp"
#include "mlp_infer.hpp"

namespace d2q37 {

constexpr int LBLOCK = 512;
constexpr int LWAVES = LBLOCK / 64;

constexpr int FQ = 128;  // fallback queue of a wavefront (circular): < 64 waiting + one tile's 64
constexpr int RS = 40;   // floats per ring slot: the 37 populations, padded to 160 bytes
constexpr int LRING_WGS = 256;  // workgroups the ring holds slots for (the persistent grid's cap)
constexpr size_t RING_WG_BYTES = (size_t)LWAVES * FQ * RS * sizeof(float);

struct LearnedLds {
    mlp::SharedWeights w;
    uint16_t X[LWAVES][mlp::WAVE_LDS_BYTES / 2];
    uint32_t fq[LWAVES][FQ];  // queued fallback sites, x * LY + r (r: slot in row x)
    double red[LWAVES][4];
};
static_assert(sizeof(LearnedLds) <= 160 * 1024, "the learned kernels' LDS must fit one compute unit");

// Plain FP32 collide of the n <= 64 queued fallback sites from queue position
// h on, one per lane: populations read from their ring slots, result stored
// at the site in dst. Every lane must call it, after the ring writes are
// visible (fence_ring).
template <class L, bool COMP, bool AUDIT>
__device__ inline void fallback_batch(const uint32_t* q, const float* ring, int h, int n, float* dst, const Geo& g,
                                      float om, double (&acc)[4])
{
    using P = PrecF32S;
    constexpr int VL = vl_of<P>();
    const int lane = mlp::lane_id();
    const bool valid = lane < n;
    const int slot = (h + (valid ? lane : 0)) & (FQ - 1);
    const uint32_t e = q[slot];
    const int fx = (int)(e / (uint32_t)g.ly), fr = (int)(e - (uint32_t)fx * (uint32_t)g.ly);
    Stencil<L, float, VL> st;
    st.setup(fx, fr, g);
    const float* sp = ring + slot * RS;
    float v[Q];
#pragma unroll
    for (int j = 0; j < Q / 4; ++j) {
        const float4 t = ((const float4*)sp)[j];
        v[4 * j] = t.x;
        v[4 * j + 1] = t.y;
        v[4 * j + 2] = t.z;
        v[4 * j + 3] = t.w;
    }
    v[Q - 1] = sp[Q - 1];
    if (valid) {
        double d[Q];
        collide_site<P, COMP>(v, om, [&](int p, float res) {
            P::template store<L::stream_stores>(st.own(dst, p, g), p, res);
            if constexpr (AUDIT) d[p] = (double)res;
        });
        if constexpr (AUDIT) audit_site(d, acc);
    }
}

// The wavefront's ring writes complete and visible to its own later reads
// (other lanes read them).
__device__ inline void fence_ring()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Queue this tile's fallback lanes (mask m of lanes with fb set; v: the
// lane's pulled populations) behind the qn entries waiting from position h,
// and, once 64 are waiting, collide the oldest 64. h, qn: wavefront-uniform.
template <class L, bool COMP, bool AUDIT>
__device__ inline void queue_fallback(uint32_t* q, float* ring, int& h, int& qn, uint64_t m, bool fb, uint32_t site,
                                      const float (&v)[Q], float* dst, const Geo& g, float om, double (&acc)[4])
{
    if (m == 0) return;
    const int lane = mlp::lane_id();
    if (fb) {
        const int slot = (h + qn + __popcll(m & ((1ull << lane) - 1ull))) & (FQ - 1);
        q[slot] = site;
        float* sp = ring + slot * RS;
#pragma unroll
        for (int j = 0; j < Q / 4; ++j)
            ((float4*)sp)[j] = float4{v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
        sp[Q - 1] = v[Q - 1];
    }
    qn += __popcll(m);
    if (qn >= 64) {
        mlp::wave_sync();
        fence_ring();
        fallback_batch<L, COMP, AUDIT>(q, ring, h, 64, dst, g, om, acc);
        h = (h + 64) & (FQ - 1);
        qn -= 64;
    }
}

// Tiles [first, end) with stride step visited by this workgroup.
struct TileWalk {
    int64_t first, end, step;
};
__device__ inline TileWalk tile_walk(int64_t ntiles)
{
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G < 8) return {b, ntiles, G};
    const int64_t xcd = b % 8, idx = b / 8;
    const int64_t nwg = (G - xcd + 7) / 8;  // workgroups dealt to this XCD
    const int64_t lo = xcd * ntiles / 8, hi = (xcd + 1) * ntiles / 8;
    return {lo + idx, hi, nwg};
}

template <bool AUDIT>
__device__ inline void finish_learned(LearnedLds& S, double (&acc)[4], unsigned long long nfb,
                                      unsigned long long nact, double* partials, unsigned long long* counts)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        atomicAdd(&counts[0], nfb);
        atomicAdd(&counts[1], nact);
    }
    if constexpr (AUDIT) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) S.red[wave][k] = acc[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double s = S.red[0][k];
                for (int w = 1; w < LWAVES; ++w) s += S.red[w][k];
                partials[4 * blockIdx.x + k] = s;
            }
        }
    }
}

// The tile loop of both learned kernels. INPLACE: the collide of the
// current buffer (src == dst, each site's own populations); otherwise the
// fused step src -> dst (pulled populations). With AUDIT,
// partials[4 * blockIdx.x ..] receive the workgroup's FP64 sums.
template <class L, bool COMP, bool AUDIT, bool INPLACE, bool FP8>
__device__ inline void learned_tiles(LearnedLds& S, const mlp::Net& gnet, const float* src, float* dst, const Geo& g,
                                     float om, float threshold, double* partials, unsigned long long* counts,
                                     float* ring_all)
{
    using P = PrecF32S;
    constexpr int VL = vl_of<P>();
    const mlp::Net net = mlp::share_weights<LBLOCK, FP8>(gnet, S.w);
    __syncthreads();
    uint16_t* X = S.X[threadIdx.x >> 6];
    uint32_t* q = S.fq[threadIdx.x >> 6];
    float* ring = ring_all + ((size_t)blockIdx.x * LWAVES + (threadIdx.x >> 6)) * (FQ * RS);
    int qh = 0, qn = 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    unsigned long long nfb = 0, nact = 0;
    const TileWalk tw = tile_walk((int64_t)g.lx * g.tpr);
    for (int64_t tile = tw.first; tile < tw.end; tile += tw.step) {
        const int xrow = (int)(tile / g.tpr);
        const int r = (int)(tile - (int64_t)xrow * g.tpr) * LBLOCK + (int)threadIdx.x;
        const bool active = r < g.ly;
        // lanes past the row end read the row's last site (valid addresses,
        // no per-load predication) and store nothing
        Stencil<L, float, VL> st;
        st.setup(xrow, active ? r : g.ly - 1, g);
        auto at = [&](int p) { return INPLACE ? st.own(src, p, g) : st.src(src, p, g); };
        // first gather: standardised network inputs (loads that keep the lines cached)
        {
            float in[Q];
#pragma unroll
            for (int p = 0; p < Q; ++p) in[p] = P::template load<false>(at(p), p);
            mlp::stage_inputs(X, net, in);
        }
        mlp::network_outputs<FP8, true>(net, X);
        // second gather: the populations for projection and relaxation
        float v[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) v[p] = P::template load<L::stream_loads>(at(p), p);
        float gh[Q];
        const mlp::Verdict vd = mlp::learned_equilibrium(v, net, X, threshold, gh);
        const bool fb = active && vd.fallback;
        // Fallback lanes store too, so that the tile writes whole lines (a
        // line with masked lanes is a partial write); their batch overwrites
        // the value later, from the ring, which also makes this safe in place.
        if (active) {
            double d[Q];
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                const float res = __builtin_fmaf(om, gh[p] - v[p], v[p]);
                P::template store<L::stream_stores>(st.own(dst, p, g), p, res);
                if constexpr (AUDIT) d[p] = (double)res;
            }
            if constexpr (AUDIT) {
                if (!fb) audit_site(d, acc);
            }
        }
        const uint64_t m = __ballot(fb);
        nfb += __popcll(m);
        nact += __popcll(__ballot(active));
        // in place, every site writes only itself, and a queued site's
        // batch reads the populations from the ring
        queue_fallback<L, COMP, AUDIT>(q, ring, qh, qn, m, fb, (uint32_t)xrow * (uint32_t)g.ly + (uint32_t)r, v, dst,
                                       g, om, acc);
        mlp::wave_sync();  // the staged rows are reused by the next tile
    }
    if (qn > 0) {
        mlp::wave_sync();
        fence_ring();
        fallback_batch<L, COMP, AUDIT>(q, ring, qh, qn, dst, g, om, acc);
    }
    finish_learned<AUDIT>(S, acc, nfb, nact, partials, counts);
}

// Fused step src -> dst with the learned collide; g.tpr counts 512-site
// tiles per row here. FP8: the network's hidden layer in e4m3.
template <class L, bool COMP, bool AUDIT, bool FP8>
__global__ __launch_bounds__(LBLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step_learned(
    const float* __restrict__ src, float* __restrict__ dst, Geo g, double omega, mlp::Net gnet, float threshold,
    double* __restrict__ partials, unsigned long long* __restrict__ counts, float* __restrict__ ring)
{
    __shared__ LearnedLds S;
    learned_tiles<L, COMP, AUDIT, false, FP8>(S, gnet, src, dst, g, (float)omega, threshold, partials, counts, ring);
}

// In-place learned collide on the current buffer (same walk).
template <class L, bool COMP, bool FP8>
__global__ __launch_bounds__(LBLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_collide_learned(
    float* __restrict__ buf, Geo g, double omega, mlp::Net gnet, float threshold,
    unsigned long long* __restrict__ counts, float* __restrict__ ring)
{
    __shared__ LearnedLds S;
    learned_tiles<L, COMP, false, true, FP8>(S, gnet, buf, buf, g, (float)omega, threshold, nullptr, counts, ring);
}

}  // namespace d2q37
