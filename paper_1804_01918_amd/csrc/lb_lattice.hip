// C ABI of the D2Q37 lattice (declared in include/lb.h): validation, the
// host-side context and the kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/lb.h"
#include "lb_kernels.hpp"
#include "lb_learned.hpp"
#include "lb_mlp_state.hpp"

using namespace d2q37;

struct lb_ctx {
    lb_config cfg;
    Geo geo;
    hipStream_t stream;
    int cur;               // buffer holding the current state
    int64_t steps;         // completed time steps
    bool half_step;        // a propagate without its collide is pending
    int64_t nblocks;       // blocks of a full-lattice launch
    double* partials;      // scratch: 4 doubles per block
    double* totals;        // scratch: 4 doubles
    unsigned long long* counts;  // scratch: learned-collide fallback and site counters
    const lb_mlp* mlp;     // learned collide, or NULL for the plain one
    float threshold;       // residual above which a site falls back
    Geo lgeo;              // geometry of the learned kernels (512-site tiles)
    int lgrid;             // their persistent grid: min(tiles, compute units, ring_wgs)
    int64_t audit_parts;   // partial sums written by the last fused audit
    bool fused_audit_valid;
    bool forced;           // nonzero body force: the collides' FORCE path
    double force[3];       // R tau gx, R tau gy, tau (1 - tau) |g|^2 / 2
    double* wall_tab;      // scratch: [2][WALL_TAB] (walls only)
    float* ring;           // scratch: fallback ring of the learned kernels, RING_WG_BYTES per workgroup
    int ring_wgs;          // workgroups it holds slots for
    int device;            // device current at lb_init (where the buffers live)
    void* static_scratch;  // that device's address of `scratch` (lb_audit_static), or NULL
    bool f16_stream_stores;  // FP16 buffers of at least STREAM_STORE_BYTES: hinted stores in lb_step
    char err[512];
};

// ---- library-owned scratch of lb_audit_static ---------------------------------
// A file-scope device array, so that callers who cannot allocate device memory
// can still audit: 4 FP64 partial sums per 256-site row tile (the same
// partials lb_audit keeps in the caller's scratch) followed by the 4 totals.
// Every device that loads the library holds its own copy until the process
// ends. Host code never passes the array's name to a kernel or a copy: it
// uses the device address that hipGetSymbolAddress returns for the current
// device, resolved once per device by lb_init.
// FP16 buffers from this size on (each) are stepped with hinted stores
// (PrecF16SN): at 2048^2 (310 MB) the cached stores are faster, at 4096^2
// (1.24 GB) the hinted ones; the GPU's last-level cache holds 256 MB.
constexpr size_t STREAM_STORE_BYTES = (size_t)512 << 20;

constexpr int64_t STATIC_AUDIT_MAX_TILES = (int64_t)1 << 18;  // 8192 x 8192 sites
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)(STATIC_AUDIT_MAX_TILES * 4 + 4) * sizeof(double);
static __device__ __align__(256) double scratch[STATIC_AUDIT_MAX_TILES * 4 + 4];

namespace {

thread_local char g_err[512];

int fail(lb_ctx* c, int code, const char* fmt, ...)
{
    char* dst = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(lb_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LB_OK;
    return fail(c, LB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int elem_bytes(int precision)
{
    switch (precision) {
        case LB_FP64: return 8;
        case LB_FP32_SHIFTED: return 4;
        case LB_FP16_SHIFTED: return 2;
        default: return 0;
    }
}

bool layout_ok(int layout) { return layout >= LB_SOA && layout <= LB_CAOSOA; }

int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// The kernels keep each lane's in-row column term as a 32-bit byte offset
// (Stencil::col): the bytes of one lattice row within one population term
// must not exceed 4 GiB. That is LY * 37 elements for AoS and CAoSoA (all
// populations of a row interleaved) and LY elements for SoA and CSoA.
bool row_bytes_ok(int32_t ly, int eb, int layout)
{
    const uint64_t per = (layout == LB_AOS || layout == LB_CAOSOA) ? (uint64_t)Q * eb : (uint64_t)eb;
    return (uint64_t)ly * per <= ((uint64_t)1 << 32);
}

// Scratch before the fallback ring (see lb_scratch_bytes), a multiple of 256.
size_t base_scratch_bytes(int32_t lx, int32_t ly)
{
    return round256((size_t)((int64_t)lx * div_up(ly, BLOCK) * 4 + 4 + 2 + 2 * WALL_TAB) * sizeof(double));
}
// Workgroups of the learned kernels' persistent grid the ring holds slots
// for: one per 512-site tile, at most LRING_WGS.
int ring_wgs_of(int32_t lx, int32_t ly)
{
    return (int)std::min<int64_t>((int64_t)lx * div_up(ly, LBLOCK), LRING_WGS);
}

// Calls f(P{}, L{}) for the runtime precision and layout.
template <class P, class F>
void with_layout(int layout, F&& f)
{
    constexpr int VL = vl_of<P>();
    switch (layout) {
        case LB_SOA: f(P{}, Layout<LAYOUT_SOA, VL>{}); break;
        case LB_AOS: f(P{}, Layout<LAYOUT_AOS, VL>{}); break;
        case LB_CSOA: f(P{}, Layout<LAYOUT_CSOA, VL>{}); break;
        default: f(P{}, Layout<LAYOUT_CAOSOA, VL>{}); break;
    }
}

template <class F>
void with_config(const lb_config& cfg, F&& f)
{
    switch (cfg.precision) {
        case LB_FP64: with_layout<PrecF64>(cfg.layout, f); break;
        case LB_FP32_SHIFTED: with_layout<PrecF32S>(cfg.layout, f); break;
        default: with_layout<PrecF16S>(cfg.layout, f); break;
    }
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

void* cur_buf(lb_ctx* c) { return c->cfg.buf[c->cur]; }
void* other_buf(lb_ctx* c) { return c->cfg.buf[c->cur ^ 1]; }

int launch_status(lb_ctx* c, const char* what) { return check_hip(c, hipGetLastError(), what); }

dim3 grid_of(const lb_ctx* c) { return dim3((unsigned)c->nblocks); }

template <typename C>
Force<C> force_of(const lb_ctx* c)
{
    return Force<C>{(C)c->force[0], (C)c->force[1], (C)c->force[2]};
}

// Walls: the emission of both walls into the current buffer's slots that
// the next pull reads from beyond them (before a propagate or step).
void launch_wall(lb_ctx* c)
{
    with_config(c->cfg, [&](auto p, auto l) {
        using P = decltype(p);
        using L = decltype(l);
        const int64_t blocks = div_up(c->geo.lx, BLOCK / 64);  // one wavefront per column
        hipLaunchKernelGGL((k_wall<P, L>), dim3((unsigned)blocks), dim3(BLOCK), 0, c->stream,
                           (typename P::T*)cur_buf(c), c->geo, (const double*)c->wall_tab);
    });
}
dim3 lgrid_of(const lb_ctx* c) { return dim3((unsigned)c->lgrid); }

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[MAX_DEVICES];
void* g_scratch_ptr[MAX_DEVICES];
hipError_t g_scratch_err[MAX_DEVICES];

// Device address of `scratch` on device `dev`, which must be current.
// Resolved on the first call per device; NULL (and *err set) on failure.
void* static_scratch_of(int dev, hipError_t* err)
{
    *err = hipSuccess;
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
        g_scratch_done[dev] = true;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

// Audit of the current buffer into `partials` (4 per tile) and `totals`
// (4), copied to out on the host; `use_fused` takes the partials of the last
// fused step, which are already in `partials`.
int audit_into(lb_ctx* c, double* partials, double* totals, bool use_fused, double out[4], const char* what)
{
    char msg[96];
    if (!use_fused) {
        with_config(c->cfg, [&](auto p, auto l) {
            using P = decltype(p);
            using L = decltype(l);
            hipLaunchKernelGGL((k_audit<P, L>), grid_of(c), dim3(BLOCK), 0, c->stream,
                               (const typename P::T*)cur_buf(c), c->geo, partials);
        });
        snprintf(msg, sizeof msg, "%s: partials", what);
        const int rc = launch_status(c, msg);
        if (rc != LB_OK) return rc;
    }
    const double n = (double)c->geo.n;
    const bool shifted = c->cfg.precision != LB_FP64;
    const double4 base = shifted ? double4{n, 0.0, 0.0, n} : double4{0.0, 0.0, 0.0, 0.0};
    const int64_t nparts = use_fused ? c->audit_parts : c->nblocks;
    hipLaunchKernelGGL(k_audit_final, dim3(1), dim3(BLOCK), 0, c->stream, (const double*)partials, nparts, base,
                       totals);
    snprintf(msg, sizeof msg, "%s: final", what);
    int rc = launch_status(c, msg);
    if (rc != LB_OK) return rc;
    snprintf(msg, sizeof msg, "%s: copy", what);
    rc = check_hip(c, hipMemcpyAsync(out, totals, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), msg);
    if (rc != LB_OK) return rc;
    snprintf(msg, sizeof msg, "%s: synchronize", what);
    rc = check_hip(c, hipStreamSynchronize(c->stream), msg);
    if (rc != LB_OK) return rc;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(out[i])) return fail(c, LB_ENONFINITE, "%s: total %d is not finite", what, i);
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lb_buffer_bytes(int32_t lx, int32_t ly, int32_t precision, int32_t layout)
{
    const int eb = elem_bytes(precision);
    if (lx < 1 || ly < 1 || eb == 0 || !layout_ok(layout)) return 0;
    const int64_t n = (int64_t)lx * ly;
    if (n >= ((int64_t)1 << 31)) return 0;
    if (!row_bytes_ok(ly, eb, layout)) return 0;
    if (layout == LB_CSOA || layout == LB_CAOSOA) {
        const int vl = 128 / eb;
        if (ly % vl != 0) return 0;
    }
    return round256((size_t)n * Q * eb);
}

size_t lb_scratch_bytes(int32_t lx, int32_t ly)
{
    if (lx < 1 || ly < 1) return 0;
    const int64_t n = (int64_t)lx * ly;
    if (n >= ((int64_t)1 << 31)) return 0;
    // one partial sum of 4 doubles per row-tiled workgroup, the 4 totals, two
    // 64-bit counters of the learned collide and the walls' table; then the
    // learned kernels' fallback ring
    return base_scratch_bytes(lx, ly) + (size_t)ring_wgs_of(lx, ly) * RING_WG_BYTES;
}

int lb_init(lb_ctx** out, const lb_config* cfg, const double* rho, const double* ux, const double* uy,
            const double* T)
{
    if (!out) return fail(nullptr, LB_EINVAL, "lb_init: out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, LB_EINVAL, "lb_init: cfg is NULL");
    const lb_config& k = *cfg;
    if (k.lx < 1 || k.ly < 1) return fail(nullptr, LB_EINVAL, "lb_init: extents %d x %d must be >= 1", k.lx, k.ly);
    if ((int64_t)k.lx * k.ly >= ((int64_t)1 << 31))
        return fail(nullptr, LB_EINVAL, "lb_init: %d x %d sites exceed 2^31 - 1", k.lx, k.ly);
    if (!(k.tau > 0.5) || !std::isfinite(k.tau))
        return fail(nullptr, LB_EINVAL, "lb_init: tau = %g must be finite and > 0.5", k.tau);
    if (elem_bytes(k.precision) == 0) return fail(nullptr, LB_EUNSUPPORTED, "lb_init: unknown precision %d", k.precision);
    if (!layout_ok(k.layout)) return fail(nullptr, LB_EUNSUPPORTED, "lb_init: unknown layout %d", k.layout);
    if (!row_bytes_ok(k.ly, elem_bytes(k.precision), k.layout))
        return fail(nullptr, LB_EUNSUPPORTED,
                    "lb_init: a row of %d sites spans more than 4 GiB per population term in layout %d", k.ly,
                    k.layout);
    const size_t bb = lb_buffer_bytes(k.lx, k.ly, k.precision, k.layout);
    if (bb == 0)
        return fail(nullptr, LB_EUNSUPPORTED, "lb_init: layout %d needs LY (%d) to be a multiple of %d", k.layout,
                    k.ly, 128 / elem_bytes(k.precision));
    for (int i = 0; i < 2; ++i)
        if (!k.buf[i] || !aligned256(k.buf[i]))
            return fail(nullptr, LB_EINVAL, "lb_init: buf[%d] is NULL or not 256-byte aligned", i);
    if (k.buf[0] == k.buf[1]) return fail(nullptr, LB_EINVAL, "lb_init: buf[0] and buf[1] must differ");
    if (!k.scratch || !aligned256(k.scratch)) return fail(nullptr, LB_EINVAL, "lb_init: scratch is NULL or misaligned");
    if (k.scratch_bytes < lb_scratch_bytes(k.lx, k.ly))
        return fail(nullptr, LB_EINVAL, "lb_init: scratch_bytes %zu < %zu", k.scratch_bytes,
                    lb_scratch_bytes(k.lx, k.ly));
    if (!rho || !ux || !uy || !T) return fail(nullptr, LB_EINVAL, "lb_init: a field pointer is NULL");
    if (!std::isfinite(k.gx) || !std::isfinite(k.gy) || std::fabs(k.gx) > 1.0 || std::fabs(k.gy) > 1.0)
        return fail(nullptr, LB_EINVAL, "lb_init: force (%g, %g) must be finite with |g| <= 1", k.gx, k.gy);
    if (k.walls != 0 && k.walls != 1) return fail(nullptr, LB_EINVAL, "lb_init: walls = %d must be 0 or 1", k.walls);
    if (k.walls && (!(k.t_bottom > 0.0) || !(k.t_top > 0.0) || !std::isfinite(k.t_bottom) || !std::isfinite(k.t_top)))
        return fail(nullptr, LB_EINVAL, "lb_init: wall temperatures (%g, %g) must be finite and > 0", k.t_bottom,
                    k.t_top);

    lb_ctx* c = new (std::nothrow) lb_ctx();
    if (!c) return fail(nullptr, LB_EINVAL, "lb_init: out of host memory");
    c->cfg = k;
    c->geo.lx = k.lx;
    c->geo.ly = k.ly;
    c->geo.n = (int64_t)k.lx * k.ly;
    c->geo.lyv = (k.layout == LB_CSOA || k.layout == LB_CAOSOA) ? k.ly / (128 / elem_bytes(k.precision)) : k.ly;
    c->stream = (hipStream_t)k.stream;
    c->cur = 0;
    c->steps = 0;
    c->half_step = false;
    c->geo.tpr = (int)div_up(k.ly, BLOCK);
    c->nblocks = (int64_t)k.lx * c->geo.tpr;
    c->partials = (double*)k.scratch;
    c->totals = c->partials + 4 * c->nblocks;
    c->counts = (unsigned long long*)(c->totals + 4);
    c->wall_tab = c->totals + 4 + 2;
    c->ring = (float*)((char*)k.scratch + base_scratch_bytes(k.lx, k.ly));
    c->ring_wgs = ring_wgs_of(k.lx, k.ly);
    c->forced = k.gx != 0.0 || k.gy != 0.0;
    c->force[0] = R * k.tau * k.gx;
    c->force[1] = R * k.tau * k.gy;
    c->force[2] = k.tau * (1.0 - k.tau) * (k.gx * k.gx + k.gy * k.gy) / 2.0;
    c->mlp = nullptr;
    c->threshold = 0.0f;
    c->lgeo = c->geo;
    c->lgrid = 1;
    c->audit_parts = c->nblocks;
    c->fused_audit_valid = false;
    c->err[0] = 0;
    c->device = -1;
    c->static_scratch = nullptr;
    c->f16_stream_stores = k.precision == LB_FP16_SHIFTED && bb >= STREAM_STORE_BYTES;
    if (hipGetDevice(&c->device) == hipSuccess) {
        hipError_t e;
        c->static_scratch = static_scratch_of(c->device, &e);
    }

    with_config(k, [&](auto p, auto l) {
        using P = decltype(p);
        using L = decltype(l);
        hipLaunchKernelGGL((k_init<P, L>), grid_of(c), dim3(BLOCK), 0, c->stream, (typename P::T*)k.buf[0],
                           c->geo, rho, ux, uy, T);
    });
    if (k.walls) hipLaunchKernelGGL(k_wall_setup, dim3(1), dim3(64), 0, c->stream, c->wall_tab, k.t_bottom, k.t_top);
    if (hipMemsetAsync(c->counts, 0, 2 * sizeof(unsigned long long), c->stream) != hipSuccess) {
        snprintf(g_err, sizeof g_err, "lb_init: clearing the counters failed");
        delete c;
        return LB_EDEVICE;
    }
    const int rc = launch_status(c, "lb_init: launch");
    if (rc != LB_OK) {
        snprintf(g_err, sizeof g_err, "%s", c->err);
        delete c;
        return rc;
    }
    *out = c;
    return LB_OK;
}

int lb_propagate(lb_ctx* c)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_propagate: ctx is NULL");
    if (c->cfg.walls) launch_wall(c);
    with_config(c->cfg, [&](auto p, auto l) {
        using P = decltype(p);
        using L = decltype(l);
        hipLaunchKernelGGL((k_propagate<P, L>), grid_of(c), dim3(BLOCK), 0, c->stream,
                           (const typename P::Word*)cur_buf(c), (typename P::Word*)other_buf(c), c->geo);
    });
    const int rc = launch_status(c, "lb_propagate");
    if (rc != LB_OK) return rc;
    c->cur ^= 1;
    c->half_step = true;
    c->fused_audit_valid = false;
    return LB_OK;
}

int lb_collide(lb_ctx* c)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_collide: ctx is NULL");
    const double omega = 1.0 / c->cfg.tau;
    const bool comp = c->cfg.compensated != 0;
    if (c->mlp) {
        const bool fp8 = c->mlp->precision == LB_MLP_FP8;
        with_layout<PrecF32S>(c->cfg.layout, [&](auto, auto l) {
            using L = decltype(l);
#define D2Q37_LCOLL(CMP, F8)                                                                                       \
    hipLaunchKernelGGL((k_collide_learned<L, CMP, F8>), lgrid_of(c), dim3(LBLOCK), 0, c->stream, (float*)cur_buf(c), \
                       c->lgeo, omega, c->mlp->net(), c->threshold, c->counts, c->ring)
            if (comp) {
                if (fp8) D2Q37_LCOLL(true, true); else D2Q37_LCOLL(true, false);
            } else {
                if (fp8) D2Q37_LCOLL(false, true); else D2Q37_LCOLL(false, false);
            }
#undef D2Q37_LCOLL
        });
    } else {
        with_config(c->cfg, [&](auto p, auto l) {
            using P = decltype(p);
            using L = decltype(l);
            const auto force = force_of<typename P::C>(c);
            auto* buf = (typename P::T*)cur_buf(c);
#define D2Q37_COLL(CMP, FRC) \
    hipLaunchKernelGGL((k_collide<P, L, CMP, FRC>), grid_of(c), dim3(BLOCK), 0, c->stream, buf, c->geo, omega, force)
            if (comp) {
                if (c->forced) D2Q37_COLL(true, true); else D2Q37_COLL(true, false);
            } else {
                if (c->forced) D2Q37_COLL(false, true); else D2Q37_COLL(false, false);
            }
#undef D2Q37_COLL
        });
    }
    const int rc = launch_status(c, "lb_collide");
    if (rc != LB_OK) return rc;
    if (c->half_step) {
        c->steps += 1;
        c->half_step = false;
    }
    c->fused_audit_valid = false;
    return LB_OK;
}

int lb_step(lb_ctx* c, int32_t nsteps)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_step: ctx is NULL");
    if (nsteps < 0) return fail(c, LB_EINVAL, "lb_step: nsteps = %d < 0", nsteps);
    if (nsteps == 0) return LB_OK;
    const double omega = 1.0 / c->cfg.tau;
    const bool comp = c->cfg.compensated != 0;
    for (int32_t s = 0; s < nsteps; ++s) {
        const bool audit = c->cfg.audit && s == nsteps - 1;
        if (c->mlp) {
            with_layout<PrecF32S>(c->cfg.layout, [&](auto, auto l) {
                using L = decltype(l);
                const float* src = (const float*)cur_buf(c);
                float* dst = (float*)other_buf(c);
                const bool fp8 = c->mlp->precision == LB_MLP_FP8;
#define D2Q37_LSTEP(CMP, AUD, F8)                                                                                  \
    hipLaunchKernelGGL((k_step_learned<L, CMP, AUD, F8>), lgrid_of(c), dim3(LBLOCK), 0, c->stream, src, dst, c->lgeo, \
                       omega, c->mlp->net(), c->threshold, c->partials, c->counts, c->ring)
#define D2Q37_LSTEP8(CMP, AUD) \
    do { if (fp8) D2Q37_LSTEP(CMP, AUD, true); else D2Q37_LSTEP(CMP, AUD, false); } while (0)
                if (comp) {
                    if (audit) D2Q37_LSTEP8(true, true); else D2Q37_LSTEP8(true, false);
                } else {
                    if (audit) D2Q37_LSTEP8(false, true); else D2Q37_LSTEP8(false, false);
                }
#undef D2Q37_LSTEP8
#undef D2Q37_LSTEP
            });
            const int rc = launch_status(c, "lb_step (learned collide)");
            if (rc != LB_OK) return rc;
            c->cur ^= 1;
            c->steps += 1;
            c->fused_audit_valid = audit;
            if (audit) c->audit_parts = c->lgrid;
            continue;
        }
        if (c->cfg.walls) launch_wall(c);
        with_config(c->cfg, [&](auto p, auto l) {
            using P = decltype(p);
            using L = decltype(l);
            const auto* src = (const typename P::T*)cur_buf(c);
            auto* dst = (typename P::T*)other_buf(c);
            const auto force = force_of<typename P::C>(c);
            auto launch = [&](auto pk) {
                using PK = decltype(pk);  // P, or its hinted-store form
#define D2Q37_STEP(CMP, AUD, FRC)                                                                                 \
    hipLaunchKernelGGL((k_step<PK, L, CMP, AUD, FRC>), grid_of(c), dim3(BLOCK), 0, c->stream, src, dst, c->geo, omega, \
                       c->partials, force)
#define D2Q37_STEP_BC(CMP, AUD) \
    do { if (c->forced) D2Q37_STEP(CMP, AUD, true); else D2Q37_STEP(CMP, AUD, false); } while (0)
                if (comp) {
                    if (audit) D2Q37_STEP_BC(true, true); else D2Q37_STEP_BC(true, false);
                } else {
                    if (audit) D2Q37_STEP_BC(false, true); else D2Q37_STEP_BC(false, false);
                }
#undef D2Q37_STEP_BC
#undef D2Q37_STEP
            };
            if constexpr (P::kind == PREC_F16S) {
                if (c->f16_stream_stores) launch(PrecF16SN{});
                else launch(P{});
            } else {
                launch(P{});
            }
        });
        const int rc = launch_status(c, "lb_step");
        if (rc != LB_OK) return rc;
        c->cur ^= 1;
        c->steps += 1;
        c->fused_audit_valid = audit;
        if (audit) c->audit_parts = c->nblocks;
    }
    return LB_OK;
}

int lb_moments(lb_ctx* c, double* rho, double* ux, double* uy, double* T)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_moments: ctx is NULL");
    if (!rho || !ux || !uy || !T) return fail(c, LB_EINVAL, "lb_moments: a field pointer is NULL");
    with_config(c->cfg, [&](auto p, auto l) {
        using P = decltype(p);
        using L = decltype(l);
        hipLaunchKernelGGL((k_moments<P, L>), grid_of(c), dim3(BLOCK), 0, c->stream,
                           (const typename P::T*)cur_buf(c), c->geo, rho, ux, uy, T);
    });
    return launch_status(c, "lb_moments");
}

int lb_get_populations(lb_ctx* c, double* f)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_get_populations: ctx is NULL");
    if (!f) return fail(c, LB_EINVAL, "lb_get_populations: f is NULL");
    with_config(c->cfg, [&](auto p, auto l) {
        using P = decltype(p);
        using L = decltype(l);
        hipLaunchKernelGGL((k_get<P, L>), grid_of(c), dim3(BLOCK), 0, c->stream, (const typename P::T*)cur_buf(c),
                           c->geo, f);
    });
    return launch_status(c, "lb_get_populations");
}

int lb_set_populations(lb_ctx* c, const double* f)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_set_populations: ctx is NULL");
    if (!f) return fail(c, LB_EINVAL, "lb_set_populations: f is NULL");
    with_config(c->cfg, [&](auto p, auto l) {
        using P = decltype(p);
        using L = decltype(l);
        hipLaunchKernelGGL((k_set<P, L>), grid_of(c), dim3(BLOCK), 0, c->stream, (typename P::T*)cur_buf(c), c->geo,
                           f);
    });
    c->fused_audit_valid = false;
    return launch_status(c, "lb_set_populations");
}

int lb_audit(lb_ctx* c, double out[4])
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_audit: ctx is NULL");
    if (!out) return fail(c, LB_EINVAL, "lb_audit: out is NULL");
    return audit_into(c, c->partials, c->totals, c->fused_audit_valid, out, "lb_audit");
}

int lb_audit_static(lb_ctx* c, double out[4])
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_audit_static: ctx is NULL");
    if (!out) return fail(c, LB_EINVAL, "lb_audit_static: out is NULL");
    if (c->nblocks > STATIC_AUDIT_MAX_TILES)
        return fail(c, LB_EINVAL,
                    "lb_audit_static: %lld row tiles of %d sites exceed the library scratch (%lld tiles, %zu bytes)",
                    (long long)c->nblocks, BLOCK, (long long)STATIC_AUDIT_MAX_TILES, STATIC_SCRATCH_BYTES);
    if (!c->static_scratch) {
        hipError_t e = hipSuccess;
        if (c->device >= 0) static_scratch_of(c->device, &e);
        return fail(c, LB_EDEVICE, "lb_audit_static: no address of the library scratch on device %d: %s", c->device,
                    hipGetErrorString(e));
    }
    double* partials = (double*)c->static_scratch;
    double* totals = partials + 4 * c->nblocks;
    return audit_into(c, partials, totals, false, out, "lb_audit_static");
}

int lb_set_surrogate(lb_ctx* c, const lb_mlp* m, double threshold)
{
    if (!c) return fail(nullptr, LB_EINVAL, "lb_set_surrogate: ctx is NULL");
    if (!m) {
        c->mlp = nullptr;
        return LB_OK;
    }
    if (c->cfg.precision != LB_FP32_SHIFTED)
        return fail(c, LB_EUNSUPPORTED, "lb_set_surrogate: the learned collide needs FP32-shifted populations");
    if (c->forced || c->cfg.walls)
        return fail(c, LB_EUNSUPPORTED, "lb_set_surrogate: the learned collide runs on periodic lattices without force");
    if (!(threshold >= 0.0) || !std::isfinite(threshold))
        return fail(c, LB_EINVAL, "lb_set_surrogate: threshold %g must be finite and >= 0", threshold);
    if ((int64_t)c->geo.lx * c->geo.ly > (int64_t)UINT32_MAX)
        return fail(c, LB_EINVAL, "lb_set_surrogate: the learned collide takes lattices of at most 2^32 - 1 sites");
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return fail(c, LB_EDEVICE, "lb_set_surrogate: cannot query the compute-unit count");
    c->lgeo = c->geo;
    c->lgeo.tpr = (int)div_up(c->geo.ly, LBLOCK);
    const int64_t tiles = (int64_t)c->geo.lx * c->lgeo.tpr;
    // one workgroup per compute unit, and no more than the ring has slots for
    c->lgrid = (int)std::min<int64_t>(std::min<int64_t>(tiles, ncu), c->ring_wgs);
    c->mlp = m;
    c->threshold = (float)threshold;
    return LB_OK;
}

int lb_surrogate_counts(lb_ctx* c, int64_t out[2])
{
    if (!c || !out) return fail(c, LB_EINVAL, "lb_surrogate_counts: NULL argument");
    unsigned long long h[2];
    int rc = check_hip(c, hipMemcpyAsync(h, c->counts, sizeof h, hipMemcpyDeviceToHost, c->stream),
                       "lb_surrogate_counts: copy");
    if (rc == LB_OK) rc = check_hip(c, hipMemsetAsync(c->counts, 0, sizeof h, c->stream), "lb_surrogate_counts: reset");
    if (rc == LB_OK) rc = check_hip(c, hipStreamSynchronize(c->stream), "lb_surrogate_counts: synchronize");
    if (rc != LB_OK) return rc;
    out[0] = (int64_t)h[0];
    out[1] = (int64_t)h[1];
    return LB_OK;
}

int lb_current_buffer(const lb_ctx* c) { return c ? c->cur : -1; }

int64_t lb_steps_done(const lb_ctx* c) { return c ? c->steps : -1; }

void lb_destroy(lb_ctx* c) { delete c; }

const char* lb_strerror(int code)
{
    switch (code) {
        case LB_OK: return "success";
        case LB_EINVAL: return "invalid argument";
        case LB_EDEVICE: return "HIP device error";
        case LB_EUNSUPPORTED: return "unsupported combination";
        case LB_ENONFINITE: return "non-finite lattice totals";
        default: return "unknown error code";
    }
}

const char* lb_last_error(const lb_ctx* c) { return c ? c->err : g_err; }

int lb_model_constants(double* r, double* w, int32_t* cvec)
{
    if (r) *r = R;
    for (int p = 0; p < Q; ++p) {
        if (w) w[p] = weight(p);
        if (cvec) {
            cvec[2 * p] = CX[p];
            cvec[2 * p + 1] = CY[p];
        }
    }
    return LB_OK;
}

int lb_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (!dst || !src || (bytes & 15u) || ((uintptr_t)dst & 15u) || ((uintptr_t)src & 15u))
        return fail(nullptr, LB_EINVAL, "lb_copy: NULL or misaligned pointer, or size not a multiple of 16");
    if (bytes == 0) return LB_OK;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = div_up(n16, (int64_t)BLOCK * COPY_UNROLL);
    if (blocks > 0x7fffffff) return fail(nullptr, LB_EINVAL, "lb_copy: %zu bytes is too large", bytes);
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(BLOCK), 0, (hipStream_t)stream, (const u32x4*)src,
                       (u32x4*)dst, n16);
    return check_hip(nullptr, hipGetLastError(), "lb_copy");
}

}  // extern "C"
