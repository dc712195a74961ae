/*
 * lb.h - C ABI of libd2q37: one D2Q37 Lattice Boltzmann time step on an
 * AMD Instinct MI355X (gfx950).
 *
 * The problem (paper: Calore, Gabbana, Schifano, Tripiccione, "Early
 * experience on using Knights Landing processors for Lattice Boltzmann
 * applications", Section 3 and Listing 1):
 *   - a periodic LX x LY lattice with 37 populations per site, each moving up
 *     to three lattice points per step (the D2Q37 model);
 *   - two copies of the populations; a time step is propagate (every
 *     population moves to the site its hop points at) followed by collide
 *     (per site: density rho, velocity u and temperature T, the model's
 *     equilibrium with perfect-gas pressure p = rho T, and relaxation);
 *   - throughput counted in lattice updates per second.
 *
 * Conventions for every call:
 *   - Return 0 (LB_OK) on success or a negative LB_E* code; lb_last_error()
 *     gives a message. No C++ exception crosses this interface.
 *   - Device pointers are plain HIP device addresses (for example from
 *     torch.empty(..., device="cuda").data_ptr()). Every device call is
 *     asynchronous on the context's stream; calls that return host data
 *     (lb_audit, lb_last_error) synchronise that stream. A device fault
 *     surfaces at the next synchronising call as LB_EDEVICE.
 *   - Ownership: the caller owns every device buffer (the two population
 *     buffers and the scratch area) and must keep them alive until
 *     lb_destroy. The library allocates no device memory; it allocates and
 *     frees only its host-side context.
 *   - Units: velocities and temperature are in thermal units (velocity in
 *     units of the reference thermal speed, T relative to the reference
 *     temperature); the lattice hop c_p corresponds to the thermal velocity
 *     xi_p = r c_p with r = 1.19697977... (see lb_model_constants).
 *   - Canonical interchange layout of populations: FP64 f[p][x][y], y
 *     contiguous (site index = LY*x + y, as in Listing 1); p follows the
 *     population order of lb_model_constants. Fields are FP64 [x][y].
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LIBD2Q37_LB_H
#define LIBD2Q37_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_Q 37

enum {
    LB_OK = 0,
    LB_EINVAL = -1,        /* bad extent, tau, pointer, alignment or size */
    LB_EDEVICE = -2,       /* a HIP call failed; see lb_last_error */
    LB_EUNSUPPORTED = -3,  /* combination of options not provided */
    LB_ENONFINITE = -4     /* the audit found NaN or Inf in the lattice totals */
};

/* Storage precision of the populations (the computation follows it):
 *   LB_FP64         f in FP64, FP64 arithmetic.
 *   LB_FP32_SHIFTED g = f - w_p (deviation from the rest state rho0 = 1)
 *                   in FP32; FP32 arithmetic; moments with compensated sums
 *                   unless lb_config.compensated = 0.
 *   LB_FP16_SHIFTED g * s_p in FP16, s_p an exact power of two near 1/w_p;
 *                   FP32 arithmetic. */
typedef enum { LB_FP64 = 0, LB_FP32_SHIFTED = 1, LB_FP16_SHIFTED = 2 } lb_precision;

/* Memory layout of the populations (paper, Section 4, Fig. 2); VL is 128
 * bytes of storage (16 FP64, 32 FP32, 64 FP16 values):
 *   LB_SOA    [p][x][y]
 *   LB_AOS    [x][y][p]
 *   LB_CSOA   [p][x][i][k]   y = i + k*(LY/VL); needs LY % VL == 0
 *   LB_CAOSOA [x][i][p][k]   same clusters, the 37 of a site index adjacent */
typedef enum { LB_SOA = 0, LB_AOS = 1, LB_CSOA = 2, LB_CAOSOA = 3 } lb_layout;

typedef struct {
    int32_t lx, ly;       /* periodic extents, >= 1 each, lx*ly < 2^31; one row of a
                             population term at most 4 GiB: ly*37*elem <= 2^32 for
                             AoS and CAoSoA, ly*elem <= 2^32 for SoA and CSoA */
    double tau;           /* BGK relaxation time in steps, > 0.5 */
    int32_t precision;    /* lb_precision */
    int32_t layout;       /* lb_layout */
    int32_t compensated;  /* FP32 moment sums of the shifted precisions: 1 = compensated
                             (TwoSum cascades), 0 = plain; FP64 ignores it */
    int32_t audit;        /* nonzero: lb_step fuses the FP64 audit sums into its last step */
    void *buf[2];         /* device, lb_buffer_bytes() each, 256-byte aligned */
    void *scratch;        /* device, >= lb_scratch_bytes(), 256-byte aligned */
    size_t scratch_bytes; /* size of scratch in bytes */
    void *stream;         /* hipStream_t to launch on; NULL = the null stream */
    /* Body force and walls (the paper's Rayleigh-Taylor setting, Section 3:
     * a fluid under gravity between a bottom and a top wall; Section 5 times
     * the extra kernels that apply them with the step). Zero-initialised
     * fields give the fully periodic lattice without force. */
    double gx, gy;        /* acceleration per time step, thermal units, finite, |g| <= 1:
                             the collide's equilibrium is taken at u + tau g and
                             T + tau (1 - tau) |g|^2 / 2, so each step adds rho g of
                             momentum and rho (u.g + |g|^2/2) of energy per site */
    int32_t walls;        /* 0: periodic in y; 1: diffuse walls at rest on the planes
                             y = -1/2 (bottom) and y = LY - 1/2 (top), x periodic: a
                             population pulled from beyond a wall is emitted by it with
                             the equilibrium at rest at the wall's temperature, the
                             density of each source column set so that the wall emits
                             the mass that left the fluid from that column towards it
                             in the same propagate (mass is conserved) */
    double t_bottom, t_top; /* wall temperatures when walls = 1: finite, > 0 */
} lb_config;

typedef struct lb_ctx lb_ctx;

/* Bytes of one population buffer (paper, Section 4: the lattice holds 37
 * populations per site, in two copies; Fig. 2 gives the layouts): 37 * lx *
 * ly elements rounded up to 256 bytes. Returns 0 if the combination is
 * invalid: an extent < 1, lx * ly >= 2^31, an unknown precision or layout,
 * ly not a multiple of VL for CSoA and CAoSoA, or a row whose bytes within
 * one population term exceed 4 GiB (ly * 37 * elem for AoS and CAoSoA,
 * ly * elem for SoA and CSoA; the kernels address a row with 32-bit byte
 * offsets). Host only; never touches the device. */
size_t lb_buffer_bytes(int32_t lx, int32_t ly, int32_t precision, int32_t layout);

/* Bytes of scratch a context of this lattice needs: the FP64 partial sums of
 * the audit (4 per 256-site row tile), its 4 totals, the two counters of
 * the learned collide, the walls' equilibrium table and their per-column
 * densities (2 * lx), then the learned collide's fallback ring (the pulled
 * populations of sites waiting for the plain collide: 160 KB for each
 * workgroup of its persistent grid, min(lx * ceil(ly / 512), 256) of
 * them); 0 for an invalid extent. Host only. */
size_t lb_scratch_bytes(int32_t lx, int32_t ly);

/* Create a context and set the populations of buf[0] to the equilibrium of
 * the FP64 device fields rho, ux, uy, T ([lx][ly] each, thermal units; read
 * only, may be freed once the stream has passed this call). The equilibrium
 * is the model's (paper, Section 3: the D2Q37 equilibrium of density rho,
 * velocity u and temperature T, with pressure p = rho T), in this build the
 * fourth-order Hermite expansion of the Maxwellian on the 37-velocity
 * quadrature. The context borrows cfg's buffers and stream until
 * lb_destroy. On error *out is NULL and nothing was launched. Validates,
 * before any device work: extents and the row-size limit of lb_config
 * (LB_EINVAL / LB_EUNSUPPORTED), tau > 0.5 and finite (LB_EINVAL), the
 * precision and layout (LB_EUNSUPPORTED), LY % VL for the clustered layouts
 * (LB_EUNSUPPORTED), non-NULL, distinct, 256-byte-aligned buffers and
 * scratch of at least lb_scratch_bytes() (LB_EINVAL), non-NULL fields
 * (LB_EINVAL), a finite force with |gx|, |gy| <= 1, walls 0 or 1 and finite
 * positive wall temperatures (LB_EINVAL). LB_EDEVICE if a launch fails. */
int lb_init(lb_ctx **out, const lb_config *cfg, const double *rho, const double *ux,
            const double *uy, const double *T);

/* Propagate (paper, Section 3; Listing 1): every population p at site s is
 * replaced by the one at s - c_p (pull gather, periodic), copied bit for bit
 * into the other buffer, which then becomes current. With walls, the
 * populations pulled from beyond a wall are the wall's emission (see
 * lb_config.walls): before the gather, each wall's densities are summed
 * from the slots of the current buffer that leave through it, and those
 * slots, which the propagate would otherwise only move across the lattice
 * to the opposite wall, receive the other wall's emission; so with walls
 * the buffer that stops being current differs from the state it held in
 * those slots only. */
int lb_propagate(lb_ctx *ctx);

/* Collide (paper, Section 3): per site, moments, equilibrium and BGK
 * relaxation f <- f - (f - f_eq)/tau, in place on the current buffer; with
 * a body force the equilibrium is taken at the shifted velocity and
 * temperature of lb_config.gx, gy. */
int lb_collide(lb_ctx *ctx);

/* nsteps time steps (paper, Section 3: a time step is propagate followed by
 * collide; Section 4 and Listing 1: two copies of the lattice, one read and
 * one written). Each step runs both in one kernel that pulls from the
 * current buffer, collides in registers and writes the other buffer, which
 * then becomes current (ping-pong). Bit-identical to nsteps x
 * (lb_propagate; lb_collide). nsteps = 0 is a no-op; LB_EINVAL for a NULL
 * context or nsteps < 0; LB_EDEVICE if a launch fails. Asynchronous. It
 * allocates nothing, synchronises nothing and issues no memset, so the
 * launches may be captured into a HIP graph on the context's stream and
 * replayed; with an even nsteps the captured buffers alternate the same way
 * on every replay. */
int lb_step(lb_ctx *ctx, int32_t nsteps);

/* Macroscopic fields of the current state (paper, Section 3: density,
 * velocity and temperature of a site, the moments the collide relaxes
 * around), in FP64 into caller-owned device arrays [lx][ly] each:
 * rho = sum f, rho u = sum f xi, rho (|u|^2 + 2 T) = sum f |xi|^2, with
 * xi = r c the thermal velocities. Under a body force these are the moments
 * of the stored (post-collision) populations; the velocity half-way through
 * the step is u - g/2. LB_EINVAL for a NULL context or array. Asynchronous. */
int lb_moments(lb_ctx *ctx, double *rho, double *ux, double *uy, double *T);

/* Current populations in the canonical FP64 layout (device [37][lx][ly],
 * caller-owned; the [p][x][y] order of Listing 1 in Section 4, converted from
 * the storage layout of Fig. 2). Shifted storage is returned as f = w_p + g
 * (exact). LB_EINVAL for a NULL context or array. Asynchronous. */
int lb_get_populations(lb_ctx *ctx, double *f);

/* Replace the current populations from canonical FP64 (device [37][lx][ly],
 * read only; same order as lb_get_populations), converted to the storage
 * layout of Fig. 2 (Section 4). Shifted storage keeps g = f - w_p rounded
 * to nearest even. Invalidates a fused audit. LB_EINVAL for a NULL context
 * or array. Asynchronous. */
int lb_set_populations(lb_ctx *ctx, const double *f);

/* Lattice totals in FP64 on the host: out = {mass, x-momentum, y-momentum,
 * energy = 1/2 sum f |xi|^2}, the quantities the collide conserves (paper,
 * Section 3: collide keeps density, momentum and energy of every site;
 * propagate only moves populations), summed in a fixed order (run to run
 * reproducible). Uses the sums fused into the last lb_step when they are
 * still current, else reduces the current buffer. Synchronises the stream.
 * Returns LB_ENONFINITE (with out filled) if any total is NaN or Inf,
 * LB_EINVAL for a NULL context or out, LB_EDEVICE on a HIP error (including
 * a fault of earlier asynchronous work). */
int lb_audit(lb_ctx *ctx, double out[4]);

/* lb_audit without the caller's scratch, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): the same totals as lb_audit, always reduced from
 * the current buffer with the same kernels, but the partial sums and totals
 * go to a scratch array inside the library (one per device, 8 MiB + 32 B,
 * held until the process ends) instead of lb_config.scratch. Allocates
 * nothing. Limit: lattices of at most 262,144 row tiles of 256 sites,
 * lx * ceil(ly / 256) <= 2^18 (8192 x 8192); larger ones return LB_EINVAL.
 * All calls on one device share that array: calls that overlap in time on
 * one device (other host threads, or other streams) race and may return
 * wrong totals. The array is fully rewritten by each call before it is read.
 * Errors as lb_audit, plus LB_EDEVICE if the array's device address could
 * not be resolved when the context was created. Synchronises the stream. */
int lb_audit_static(lb_ctx *ctx, double out[4]);

/* Index (0 or 1) of the buffer holding the current state. */
int lb_current_buffer(const lb_ctx *ctx);

/* Number of time steps applied so far (propagate + collide pairs count as one
 * after the collide). */
int64_t lb_steps_done(const lb_ctx *ctx);

void lb_destroy(lb_ctx *ctx);

const char *lb_strerror(int code);
const char *lb_last_error(const lb_ctx *ctx);

/* The library's model constants (host): r, the weights w[37] and the hops
 * c[37][2] in the library's population order. Any pointer may be NULL. */
int lb_model_constants(double *r, double *w, int32_t *c);

/* Streaming device copy of `bytes` (multiple of 16, 16-byte aligned
 * pointers) on `stream`: the reference for achievable HBM bandwidth. */
int lb_copy(void *dst, const void *src, size_t bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Learned collide. The paper's collide (Section 3) computes the equilibrium
 * from the moments in closed form; this option replaces that equilibrium by
 * a small network evaluated on the matrix cores:
 *   - input z = g / w_p (shifted populations of a site), standardised;
 *   - MLP 37 -> 128 -> 128 -> 37 with GELU (tanh form), FP32 accumulation,
 *     operands in the precision lb_mlp_set_precision selects (BF16 first
 *     layer, binary16 hidden layers by default); trained in BF16. Its
 *     output y (de-standardised) is the part of the
 *     equilibrium that the conserved moments do not fix: g_hat = P(g) + d -
 *     P(d) with d = w_p y and P the orthogonal projection (1/w inner
 *     product) onto w * {1, xi_x, xi_y, xi^2 - 2}, so mass, momentum and
 *     energy are those of g;
 *   - a site falls back to the plain collide when the deviation of g_hat's
 *     stress and heat flux from their equilibrium values of (rho, u, T)
 *     exceeds a threshold, or when (rho, |u|, T) leaves the training box
 *     [0.9, 1.1] x [0, 0.1] x [0.9, 1.1].
 * Training pairs (pre, post) come from the plain FP32 collide of seeded
 * random equilibria plus 1e-3 w_p N(0, 1) perturbations; the network is
 * trained with Adam on the target (g_eq - P(pre)) / w_p, g_eq = pre + tau
 * (post - pre). Pair arrays are device FP32 [n][37] of shifted populations.
 * Parameters travel as the packed FP32 vector W1[128][37], b1[128],
 * W2[128][128], b2[128], W3[37][128], b3[37] (26149 values); the
 * standardisation as FP32 [4][37]: mean z, sd z, mean y, sd y.
 * ------------------------------------------------------------------------- */
typedef struct lb_mlp lb_mlp;

/* Number of packed parameters (26149). */
size_t lb_mlp_param_count(void);

/* Bytes of device workspace for a network trained with batches of at most
 * max_batch pairs (a positive multiple of 32); 0 if invalid. */
size_t lb_mlp_workspace_bytes(int32_t max_batch);

/* Create a network in a caller-owned, 256-byte-aligned device workspace,
 * launching on `stream`. Parameters start at zero, standardisation at the
 * identity. */
int lb_mlp_create(lb_mlp **out, void *workspace, size_t bytes, int32_t max_batch, void *stream);
void lb_mlp_destroy(lb_mlp *m);
const char *lb_mlp_last_error(const lb_mlp *m);

/* Xavier-uniform weights and zero biases; the weight with packed index i
 * draws U from Philox4x32-10 counter (i, 0, 0xFFFFFFFF, 0), key (seed mod
 * 2^32, seed div 2^32): a (2U - 1), a = sqrt(6 / (fan_in + fan_out)), U the
 * odd multiple of 2^-24 formed from the top 23 bits of the first output word.
 * Resets the optimiser. */
int lb_mlp_init(lb_mlp *m, uint64_t seed);

/* Host FP32 packed parameters in/out (set also resets the optimiser). */
int lb_mlp_set_params(lb_mlp *m, const float *host_params);
int lb_mlp_get_params(lb_mlp *m, float *host_params);

/* Host FP32 [4][37] standardisation in/out; standard deviations > 0. */
int lb_mlp_set_normalization(lb_mlp *m, const float *host_norm);
int lb_mlp_get_normalization(lb_mlp *m, float *host_norm);

/* Mean and (population) standard deviation of z and of the target y over n
 * device pairs, summed in FP64 in a fixed order; deviations below 1e-12
 * become 1. */
int lb_mlp_fit_normalization(lb_mlp *m, const float *pre, const float *post, int64_t n, double tau);

/* Gradient of the mean squared error (over the n pairs and 37 outputs) at
 * the current parameters, for the first n device pairs (n a multiple of 32,
 * <= max_batch); host outputs. */
int lb_mlp_gradient(lb_mlp *m, const float *pre, const float *post, int32_t n, double tau, float *host_grad,
                    double *host_loss);

/* Minibatch Adam (beta 0.9, 0.999, eps 1e-8) with learning rate
 * lr * (1 + cos(pi s / S)) / 2 at step s of S = epochs * (n / batch).
 * Epoch e visits pair (a i + c) mod n at position i, with (a, c) from
 * Philox4x32-10 counter (e, 0, 0xFFFFFFFE, 0), key as for lb_mlp_init: a =
 * first word mod n moved up to the next value coprime with n (1 if 0,
 * wrapping to 1 at n), c = second word mod n; the n mod batch tail of each
 * epoch is skipped. max_steps > 0 stops early. host_epoch_loss (may be
 * NULL) receives the mean batch loss of each epoch. */
int lb_mlp_train(lb_mlp *m, const float *pre, const float *post, int64_t n, double tau, int32_t batch,
                 int32_t epochs, float lr, uint64_t seed, int64_t max_steps, double *host_epoch_loss);

/* Precision of the network's inference (the learned collide and
 * lb_mlp_equilibrium; training is always BF16 with FP32 accumulation):
 *   LB_MLP_F16   the first layer BF16 x BF16 -> FP32; the hidden
 *                activations in binary16 (IEEE half), their GELU evaluated
 *                in binary16 arithmetic, one rounding to nearest even per
 *                operation (see lb_mlp_gelu16); the last two layers
 *                binary16 x binary16 -> FP32 (the default);
 *   LB_MLP_FP8   the hidden 128 x 128 layer in FP8 (e4m3, the OCP variant
 *                without infinities): its inputs, the first layer's GELU
 *                outputs, scaled by 16, and its weights, scaled by 2^aw
 *                with aw the exponent that puts max |W2| in [128, 256),
 *                both rounded to nearest even, products accumulated in
 *                FP32 by the FP8 matrix instructions; the first and last
 *                layers stay BF16. A scaled activation beyond 448 becomes
 *                NaN and its site falls back to the plain collide.
 * lb_mlp_set_precision makes the FP8 copies from the current parameters
 * (again after every lb_mlp_init, _set_params and _train while FP8 is set).
 * LB_EINVAL for a NULL network or an unknown precision. (Not in the paper:
 * a lower-precision variant of the learned collide.) */
enum { LB_MLP_F16 = 0, LB_MLP_FP8 = 1 };
int lb_mlp_set_precision(lb_mlp *m, int32_t precision);
/* The network's inference precision (LB_MLP_F16 or LB_MLP_FP8), or
 * LB_EINVAL for a NULL network. Host only. */
int lb_mlp_get_precision(const lb_mlp *m);

/* The activation of the LB_MLP_F16 form on n device binary16 values x (bit
 * patterns) into y: gelu(x) = x / (1 + 2^(x (K1 x^2 + K2))), with K1 =
 * -2 log2(e) c A and K2 = -2 log2(e) c (c = sqrt(2 / pi), A = 0.044715: the
 * tanh form of GELU) rounded to binary16, and every operation (the square,
 * the fused K1 product and K2 sum, the product with x, the power of two,
 * the sum with 1, the reciprocal, the last product) rounded to nearest even
 * in binary16; the same instructions the learned collide runs. For
 * checking the arithmetic against a host evaluation. Asynchronous on
 * `stream`; LB_EINVAL for NULL pointers or n < 0. (Not in the paper.) */
int lb_mlp_gelu16(const uint16_t *x, uint16_t *y, int64_t n, void *stream);

/* Learned equilibrium g_hat of n device sites pre[n][37] (plain equilibrium
 * where the verdict is fallback); residual[n] (FP32) and fallback[n] (int32,
 * 1 = fallback) may be NULL. Device outputs. */
int lb_mlp_equilibrium(lb_mlp *m, const float *pre, int64_t n, float threshold, float *geq, float *residual,
                       int32_t *fallback);

/* n training pairs (device FP32 [n][37] each) from `seed`: pair k draws from
 * Philox4x32-10 key (seed mod 2^32, seed div 2^32), counters (k mod 2^32,
 * k div 2^32, j, 0), j = 0..10 (44 words w): rho = 0.9 + 0.2 U(w0), u = 0.1
 * sqrt(U(w1)) (cos, sin)(2 pi U(w2)), T = 0.9 + 0.2 U(w3), Box-Muller normals
 * n[2q], n[2q+1] from (U(w[4+2q]), U(w[5+2q])); pre = g_eq(rho, u, T) +
 * 1e-3 w_p n_p, post = the FP32 collide (relaxation time tau) of pre. */
int lb_pairgen(float *pre, float *post, int64_t n, uint64_t seed, double tau, void *stream);

/* Use the network for the collide of an FP32-shifted lattice (fused step and
 * lb_collide); NULL returns to the plain collide. The network must outlive
 * its use. Sites with residual > threshold (or outside the training box)
 * fall back to the plain FP32 collide; with threshold 0 every site does and
 * the step equals the plain FP32 step bit for bit. Errors: LB_EUNSUPPORTED
 * for FP64 or FP16 storage, or for a lattice with walls or a body force;
 * LB_EINVAL for a negative or non-finite threshold
 * or a lattice of more than 2^32 - 1 sites; LB_EDEVICE if the device cannot
 * be queried. No device memory is allocated. (Not in the paper: the learned
 * collide is an addition to its method.) */
int lb_set_surrogate(lb_ctx *ctx, const lb_mlp *m, double threshold);

/* {fallback sites, collided sites} accumulated by the learned collide since
 * the previous call (host; synchronises and resets). */
int lb_surrogate_counts(lb_ctx *ctx, int64_t out[2]);

#ifdef __cplusplus
}
#endif

#endif /* LIBD2Q37_LB_H */
