// Population storage: precision traits and the four memory layouts of the
// paper (Section 4, Fig. 2): AoS, SoA, CSoA and CAoSoA.
//
// A lattice of LX x LY sites is enumerated by "slots" 0 .. LX*LY-1 in
// storage order of one population plane; a thread owns one slot. Layouts:
//   SoA    addr = p*N + x*LY + y
//   AoS    addr = (x*LY + y)*37 + p
//   CSoA   addr = p*N + x*LY + i*VL + k          with y = i + k*LYV, LYV = LY/VL
//   CAoSoA addr = ((x*LYV + i)*37 + p)*VL + k    (same cluster index (i, k))
// In the clustered layouts the VL values of a cluster are taken LYV apart in
// y (the paper's CSoA); CAoSoA stores the 37 clusters of the same (x, i)
// back to back. VL is fixed at 128 bytes of storage: one cluster is one
// 128-byte line, so a y-hop of a cluster is an aligned line move, and
// consecutive lanes of a wavefront touch consecutive addresses.
//
// Every address is split as rowoff[cx] + coloff[cy] + pterm(p) so that the
// 37 pulled addresses of a site cost one add each after 7 + 7 setup terms.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

#include "lb_model.hpp"

namespace d2q37 {

// Population traffic is streamed: each value is read once and written once
// per step, so loads and stores carry the non-temporal hint (set either
// macro to 0 to build without it).
#ifndef D2Q37_NT_STORES
#define D2Q37_NT_STORES 1
#endif
#ifndef D2Q37_NT_LOADS
#define D2Q37_NT_LOADS 1
#endif

template <typename T, bool NT = true>
__device__ inline void st_stream(T* a, T v)
{
#if D2Q37_NT_STORES
    if constexpr (NT) __builtin_nontemporal_store(v, a);
    else *a = v;
#else
    *a = v;
#endif
}

template <typename T, bool NT = true>
__device__ inline T ld_stream(const T* a)
{
#if D2Q37_NT_LOADS
    if constexpr (NT) return __builtin_nontemporal_load(a);
    else return *a;
#else
    return *a;
#endif
}

enum LayoutKind : int { LAYOUT_SOA = 0, LAYOUT_AOS = 1, LAYOUT_CSOA = 2, LAYOUT_CAOSOA = 3 };
enum PrecisionKind : int { PREC_F64 = 0, PREC_F32S = 1, PREC_F16S = 2 };

struct Geo {
    int lx, ly;   // extents, x outer
    int lyv;      // LY / VL for clustered layouts (else LY)
    int tpr;      // workgroups per lattice row: ceil(LY / block)
    int64_t n;    // number of sites
};

// ---- precision traits --------------------------------------------------

// Plain FP64 populations f.
struct PrecF64 {
    static constexpr int kind = PREC_F64;
    using T = double;      // storage
    using C = double;      // compute
    using Word = uint64_t; // bit-copy word
    static constexpr bool shifted = false;
    template <bool NT = true>
    __device__ static C load(const T* a, int /*p*/) { return ld_stream<T, NT>(a); }
    template <bool NT = true>
    __device__ static void store(T* a, int /*p*/, C v) { st_stream<T, NT>(a, v); }
};

// Shifted deviations g = f - w in FP32.
struct PrecF32S {
    static constexpr int kind = PREC_F32S;
    using T = float;
    using C = float;
    using Word = uint32_t;
    static constexpr bool shifted = true;
    template <bool NT = true>
    __device__ static C load(const T* a, int /*p*/) { return ld_stream<T, NT>(a); }
    template <bool NT = true>
    __device__ static void store(T* a, int /*p*/, C v) { st_stream<T, NT>(a, v); }
};

// Shifted deviations stored as FP16 of g * s_p (s_p an exact power of two),
// computed in FP32. Storage holds raw FP16 bit patterns.
struct PrecF16S {
    static constexpr int kind = PREC_F16S;
    using T = uint16_t;
    using C = float;
    using Word = uint16_t;
    static constexpr bool shifted = true;
    __device__ static float scale(int p) { return S16[shell_of_c2(c2_of(p))]; }
    template <bool NT = true>
    __device__ static C load(const T* a, int p)
    {
        return __half2float(__ushort_as_half(ld_stream<T, NT>(a))) * (1.0f / scale(p));
    }
    // Stores never take the streaming hint: a wavefront's 2-byte stores
    // fill only 128 bytes per instruction, and without the hint the cache
    // merges neighbouring ones into whole lines before they go to HBM (the
    // fused step runs 9 % faster than with the hint).
    template <bool NT = true>
    __device__ static void store(T* a, int p, C v)
    {
        st_stream<T, false>(a, (uint16_t)__half_as_ushort(__float2half_rn(v * scale(p))));
    }
};

// The same storage with the streaming hint on the fused step's stores, for
// lattices whose buffers are far larger than the GPU's last-level cache:
// there a cached store buys no reuse before the line is evicted, and the
// hinted stores ran 4 % faster at 4096^2 and 8192^2 (at 2048^2, 310 MB per
// buffer, the cached ones are 8 % faster).
struct PrecF16SN : PrecF16S {
    template <bool NT = true>
    __device__ static void store(T* a, int p, C v)
    {
        st_stream<T, NT>(a, (uint16_t)__half_as_ushort(__float2half_rn(v * scale(p))));
    }
};

template <class P>
constexpr int vl_of() { return 128 / (int)sizeof(typename P::T); }

// ---- layout indexers -----------------------------------------------------

__device__ inline int wrap_periodic(int v, int L)
{
    while (v < 0) v += L;
    while (v >= L) v -= L;
    return v;
}

template <int LK, int VL>
struct Layout {
    static constexpr int kind = LK;
    static constexpr bool clustered = (LK == LAYOUT_CSOA || LK == LAYOUT_CAOSOA);
    // In AoS the 37 loads (stores) of a wavefront touch the same lines at a
    // 37-element lane stride, so the lines must stay cached between them: no
    // streaming hint on its accesses.
    static constexpr bool stream_loads = (LK != LAYOUT_AOS);
    static constexpr bool stream_stores = (LK != LAYOUT_AOS);

    // Population term of the address.
    __device__ static int64_t pterm(int p, const Geo& g)
    {
        if constexpr (LK == LAYOUT_SOA || LK == LAYOUT_CSOA) return (int64_t)p * g.n;
        else if constexpr (LK == LAYOUT_AOS) return p;
        else return (int64_t)p * VL;
    }
    // Row term for storage row x.
    __device__ static int64_t rowoff(int x, const Geo& g)
    {
        if constexpr (LK == LAYOUT_SOA || LK == LAYOUT_CSOA) return (int64_t)x * g.ly;
        else return (int64_t)x * g.ly * Q;
    }
    // Column term for in-row position (SoA/AoS: y; clustered: cluster i, lane k).
    __device__ static int64_t coloff(int y_or_i, int k)
    {
        if constexpr (LK == LAYOUT_SOA) return y_or_i;
        else if constexpr (LK == LAYOUT_AOS) return (int64_t)y_or_i * Q;
        else if constexpr (LK == LAYOUT_CSOA) return (int64_t)y_or_i * VL + k;
        else return (int64_t)y_or_i * (Q * VL) + k;
    }
};

// A thread's site and the 7 + 7 address terms of the pulled sources.
// Launches cover one lattice row x per workgroup (grid = row tiles x rows),
// so x and the row terms are uniform across the workgroup and live in scalar
// registers; only the in-row column terms (byte offsets below 4 GiB) are
// per lane.
template <class L, class T, int VL>
struct Stencil {
    int x, y;
    int64_t row[7];     // element offset of row x - cx (uniform), index cx + 3
    uint32_t col[7];    // byte offset within the row for cy, index cy + 3

    // r: position of the thread's slot within row x (0 <= r < LY).
    __device__ void setup(int xrow, int r, const Geo& g)
    {
        x = xrow;
        int i = r, k = 0;
        if constexpr (L::clustered) {
            i = r / VL;
            k = r - i * VL;
            y = i + k * g.lyv;
        } else {
            y = r;
        }
#pragma unroll
        for (int c = -3; c <= 3; ++c) row[c + 3] = L::rowoff(wrap_periodic(x - c, g.lx), g);
#pragma unroll
        for (int c = -3; c <= 3; ++c) {
            if constexpr (L::clustered) {
                int is = i - c, ks = k;
                while (is < 0) { is += g.lyv; --ks; }
                while (is >= g.lyv) { is -= g.lyv; ++ks; }
                while (ks < 0) ks += VL;
                while (ks >= VL) ks -= VL;
                col[c + 3] = (uint32_t)(L::coloff(is, ks) * (int64_t)sizeof(T));
            } else {
                col[c + 3] = (uint32_t)(L::coloff(wrap_periodic(y - c, g.ly), 0) * (int64_t)sizeof(T));
            }
        }
    }
    // Element p pulled from (x - cx_p, y - cy_p): uniform base + lane offset.
    __device__ const T* src(const T* base, int p, const Geo& g) const
    {
        const T* b = base + (L::pterm(p, g) + row[CX[p] + 3]);
        return (const T*)((const char*)b + col[CY[p] + 3]);
    }
    // Element p at the thread's own site.
    __device__ T* own(T* base, int p, const Geo& g) const
    {
        T* b = base + (L::pterm(p, g) + row[3]);
        return (T*)((char*)b + col[3]);
    }
    __device__ const T* own(const T* base, int p, const Geo& g) const
    {
        const T* b = base + (L::pterm(p, g) + row[3]);
        return (const T*)((const char*)b + col[3]);
    }
};

// Element p of site (x, y) in any layout (y -> cluster (i, k) for the
// clustered ones); used where a thread visits sites one at a time.
template <class L, int VL, class T>
__device__ inline const T* site_ptr(const T* base, int x, int y, int p, const Geo& g)
{
    int i = y, k = 0;
    if constexpr (L::clustered) {
        k = y / g.lyv;
        i = y - k * g.lyv;
    }
    return base + (L::pterm(p, g) + L::rowoff(x, g) + L::coloff(i, k));
}

// Blocks are dealt to the 8 XCDs round-robin; remap so that each XCD works
// on one contiguous range of tiles (its L2 then holds the lines shared by
// neighbouring tiles). Bijective for any block count.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb)
{
    constexpr int NXCD = 8;
    const int64_t per = nb / NXCD, rem = nb % NXCD;
    const int64_t xcd = b % NXCD, idx = b / NXCD;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Site of a thread in a row-tiled launch of LX * tpr workgroups: the block
// index is remapped per XCD, then split into (row x, tile t of the row); the
// thread's in-row position is t * block + lane. Returns false for lanes past
// the row's end.
template <int BLOCK_>
__device__ inline bool row_tile_site(const Geo& g, int& xrow, int& r, int64_t& tile_id)
{
    tile_id = xcd_tile(blockIdx.x, gridDim.x);
    xrow = (int)(tile_id / g.tpr);
    const int t = (int)(tile_id - (int64_t)xrow * g.tpr);
    r = t * BLOCK_ + (int)threadIdx.x;
    return r < g.ly;
}

}  // namespace d2q37
