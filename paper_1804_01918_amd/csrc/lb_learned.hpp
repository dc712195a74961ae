// Lattice kernels of the learned collide (FP32-shifted storage): the fused
// step and the in-place collide with the network's equilibrium, falling back
// per site to the plain FP32 collide; fallback and site counts are
// accumulated in two 64-bit counters.
#pragma once

#include "lb_kernels.hpp"
#include "mlp_infer.hpp"

namespace d2q37 {

__device__ inline void count_sites(bool fallback, bool active, unsigned long long* counts)
{
    const unsigned long long mfb = __ballot(fallback), mact = __ballot(active);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counts[0], (unsigned long long)__popcll(mfb));
        atomicAdd(&counts[1], (unsigned long long)__popcll(mact));
    }
}

// Fused step src -> dst with the learned collide. Every wavefront runs the
// network (inactive lanes carry zeros), so no lane returns early.
template <class L, bool COMP, bool AUDIT>
__global__ __launch_bounds__(BLOCK) void k_step_learned(const float* __restrict__ src, float* __restrict__ dst, Geo g,
                                                        double omega, mlp::Net net, float threshold,
                                                        double* __restrict__ partials,
                                                        unsigned long long* __restrict__ counts)
{
    using P = PrecF32S;
    D2Q37_SITE(P, L);
    __shared__ uint16_t lds[BLOCK / 64][mlp::WAVE_LDS_BYTES / 2];
    float v[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) v[p] = active ? P::template load<L::stream_loads>(st.src(src, p, g), p) : 0.0f;
    float ghat[Q];
    const mlp::Verdict vd = mlp::learned_equilibrium(v, net, lds[threadIdx.x >> 6], threshold, ghat);
    const bool fb = active && vd.fallback;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        double d[Q];
        auto store = [&](int p, float r) {
            P::template store<L::stream_stores>(st.own(dst, p, g), p, r);
            if constexpr (AUDIT) d[p] = (double)r;
        };
        const float om = (float)omega;
        if (fb) {
            collide_site<P, COMP>(v, om, store);
        } else {
#pragma unroll
            for (int p = 0; p < Q; ++p) store(p, __builtin_fmaf(om, ghat[p] - v[p], v[p]));
        }
        if constexpr (AUDIT) audit_site(d, acc);
    }
    count_sites(fb, active, counts);
    if constexpr (AUDIT) block_reduce4(acc, partials + 4 * tile);
}

// In-place learned collide on the current buffer.
template <class L, bool COMP>
__global__ __launch_bounds__(BLOCK) void k_collide_learned(float* __restrict__ buf, Geo g, double omega, mlp::Net net,
                                                           float threshold, unsigned long long* __restrict__ counts)
{
    using P = PrecF32S;
    D2Q37_SITE(P, L);
    __shared__ uint16_t lds[BLOCK / 64][mlp::WAVE_LDS_BYTES / 2];
    float v[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) v[p] = active ? P::template load<L::stream_loads>(st.own(buf, p, g), p) : 0.0f;
    float ghat[Q];
    const mlp::Verdict vd = mlp::learned_equilibrium(v, net, lds[threadIdx.x >> 6], threshold, ghat);
    const bool fb = active && vd.fallback;
    if (active) {
        auto store = [&](int p, float r) { P::template store<L::stream_stores>(st.own(buf, p, g), p, r); };
        const float om = (float)omega;
        if (fb) {
            collide_site<P, COMP>(v, om, store);
        } else {
#pragma unroll
            for (int p = 0; p < Q; ++p) store(p, __builtin_fmaf(om, ghat[p] - v[p], v[p]));
        }
    }
    count_sites(fb, active, counts);
}

}  // namespace d2q37
