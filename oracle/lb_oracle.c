/*
 * Plain FP64 CPU oracle for one D2Q37 Lattice Boltzmann time step.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it to judge the GPU library. The GPU library shares no
 * code, header or table with this file.
 *
 * What it computes (paper, Section 3 "Lattice Boltzmann Methods" and
 * Listing 1):
 *   - a lattice of LX x LY sites, periodic in both directions, 37 populations
 *     per site; populations are stored as f[p][x][y] with y contiguous,
 *     the indexing of Listing 1 (site index = LY * x + y);
 *   - one time step = propagate, then collide;
 *   - propagate moves every population along its lattice hop; written as a
 *     pull, the value arriving at site s is read from s - c_p (Listing 1 reads
 *     prv at idx + OFF[p], with OFF[p] the address of the hop's source);
 *   - collide is site-local: moments rho, u, T, the equilibrium, and a
 *     relaxation towards it.
 * The paper does not print the equilibrium or the collision operator; the
 * readings used here are
 *   - equilibrium: the Maxwellian of density rho, velocity u and
 *     temperature T, expanded in tensor Hermite polynomials of the unit
 *     Gaussian and truncated after fourth order,
 *       f_eq_i = w_i rho sum_{n=0..4} a^(n)(u,T) : H^(n)(xi_i) / n!,
 *     whose discrete pressure is p = rho T (the perfect-gas law the paper
 *     says the model enforces);
 *   - collide: single-relaxation-time BGK, f_i <- f_i - (f_i - f_eq_i) / tau.
 * Velocities are in thermal units xi_i = r c_i (the caller passes xi and the
 * weights w, both from the quadrature solve in lattice.py).
 *
 * Plain loops, no blocking, fusion or reordering: each function follows the
 * definition as written above. The loops over lattice columns x of init,
 * propagate and collide may run on several host threads (OpenMP, for the
 * all-core CPU baseline): every site's result is computed by the same code
 * from the same inputs whichever thread runs it, so the result does not
 * depend on the thread count. The audit sums stay on one thread, in order.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define Q 37
#define DIM 2

/* Host threads of the column loops; 1 unless orc_set_threads is called. */
static int orc_threads = 1;

void orc_set_threads(int n) { orc_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return orc_threads; }

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* Tensor Hermite polynomials H^(1..4) of the unit Gaussian in 2 dimensions. */
static void hermite_tensors(const double xi[DIM], double H1[DIM], double H2[DIM][DIM],
                            double H3[DIM][DIM][DIM], double H4[DIM][DIM][DIM][DIM])
{
    for (int a = 0; a < DIM; ++a) {
        H1[a] = xi[a];
        for (int b = 0; b < DIM; ++b) {
            H2[a][b] = xi[a] * xi[b] - kd(a, b);
            for (int c = 0; c < DIM; ++c) {
                H3[a][b][c] = xi[a] * xi[b] * xi[c]
                            - (xi[a] * kd(b, c) + xi[b] * kd(a, c) + xi[c] * kd(a, b));
                for (int d = 0; d < DIM; ++d) {
                    H4[a][b][c][d] = xi[a] * xi[b] * xi[c] * xi[d]
                        - (xi[a] * xi[b] * kd(c, d) + xi[a] * xi[c] * kd(b, d)
                           + xi[a] * xi[d] * kd(b, c) + xi[b] * xi[c] * kd(a, d)
                           + xi[b] * xi[d] * kd(a, c) + xi[c] * xi[d] * kd(a, b))
                        + (kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c));
                }
            }
        }
    }
}

/* Hermite coefficients, per unit density, of the Maxwellian with velocity u
 * and temperature T (reference temperature 1): with t = T - 1,
 *   a1 = u, a2 = uu + t I, a3 = uuu + t sym(u I), a4 = uuuu + t sym(uu I) + t^2 sym(I I). */
static void maxwell_coefficients(const double u[DIM], double T, double A1[DIM], double A2[DIM][DIM],
                                 double A3[DIM][DIM][DIM], double A4[DIM][DIM][DIM][DIM])
{
    const double t = T - 1.0;
    for (int a = 0; a < DIM; ++a) {
        A1[a] = u[a];
        for (int b = 0; b < DIM; ++b) {
            A2[a][b] = u[a] * u[b] + t * kd(a, b);
            for (int c = 0; c < DIM; ++c) {
                A3[a][b][c] = u[a] * u[b] * u[c]
                            + t * (u[a] * kd(b, c) + u[b] * kd(a, c) + u[c] * kd(a, b));
                for (int d = 0; d < DIM; ++d) {
                    A4[a][b][c][d] = u[a] * u[b] * u[c] * u[d]
                        + t * (u[a] * u[b] * kd(c, d) + u[a] * u[c] * kd(b, d)
                               + u[a] * u[d] * kd(b, c) + u[b] * u[c] * kd(a, d)
                               + u[b] * u[d] * kd(a, c) + u[c] * u[d] * kd(a, b))
                        + t * t * (kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c));
                }
            }
        }
    }
}

/* Equilibrium of one site: feq[i] for i < 37. xi is (37, 2) row-major. */
void orc_feq_site(const double *xi, const double *w, double rho, double ux, double uy, double T,
                  double *feq)
{
    double u[DIM] = {ux, uy};
    double A1[DIM], A2[DIM][DIM], A3[DIM][DIM][DIM], A4[DIM][DIM][DIM][DIM];
    maxwell_coefficients(u, T, A1, A2, A3, A4);
    for (int i = 0; i < Q; ++i) {
        double H1[DIM], H2[DIM][DIM], H3[DIM][DIM][DIM], H4[DIM][DIM][DIM][DIM];
        hermite_tensors(&xi[DIM * i], H1, H2, H3, H4);
        double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
        for (int a = 0; a < DIM; ++a) {
            s1 += A1[a] * H1[a];
            for (int b = 0; b < DIM; ++b) {
                s2 += A2[a][b] * H2[a][b];
                for (int c = 0; c < DIM; ++c) {
                    s3 += A3[a][b][c] * H3[a][b][c];
                    for (int d = 0; d < DIM; ++d) s4 += A4[a][b][c][d] * H4[a][b][c][d];
                }
            }
        }
        feq[i] = w[i] * rho * (1.0 + s1 + s2 / 2.0 + s3 / 6.0 + s4 / 24.0);
    }
}

/* Moments of one site: rho = sum f, rho u = sum f xi, rho (u.u + 2 T) = sum f xi.xi. */
void orc_moments_site(const double *f, const double *xi, double *rho, double *ux, double *uy,
                      double *T)
{
    double m0 = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double x = xi[DIM * i], y = xi[DIM * i + 1];
        m0 += f[i];
        jx += f[i] * x;
        jy += f[i] * y;
        e += f[i] * (x * x + y * y);
    }
    const double vx = jx / m0, vy = jy / m0;
    *rho = m0;
    *ux = vx;
    *uy = vy;
    *T = (e / m0 - (vx * vx + vy * vy)) / DIM;
}

/* BGK collision of one site, in place. */
void orc_collide_site(const double *xi, const double *w, double tau, double *f)
{
    double rho, ux, uy, T, feq[Q];
    orc_moments_site(f, xi, &rho, &ux, &uy, &T);
    orc_feq_site(xi, w, rho, ux, uy, T, feq);
    for (int i = 0; i < Q; ++i) f[i] = f[i] - (f[i] - feq[i]) / tau;
}

static size_t at(int p, int x, int y, int lx, int ly)
{
    return ((size_t)p * (size_t)lx + (size_t)x) * (size_t)ly + (size_t)y;
}

static int wrap(long v, int n)
{
    long r = v % n;
    return (int)(r < 0 ? r + n : r);
}

/* f := f_eq(rho, u, T) on every site. Fields are [lx][ly]. */
void orc_init(int lx, int ly, const double *xi, const double *w, const double *rho,
              const double *ux, const double *uy, const double *T, double *f)
{
#pragma omp parallel for num_threads(orc_threads) schedule(static)
    for (int x = 0; x < lx; ++x)
        for (int y = 0; y < ly; ++y) {
            double feq[Q];
            const size_t s = (size_t)x * ly + y;
            orc_feq_site(xi, w, rho[s], ux[s], uy[s], T[s], feq);
            for (int p = 0; p < Q; ++p) f[at(p, x, y, lx, ly)] = feq[p];
        }
}

/* Pull propagate: dst[p][x][y] = src[p][x - cx_p][y - cy_p], periodic. c is (37, 2). */
void orc_propagate(int lx, int ly, const int64_t *c, const double *src, double *dst)
{
#pragma omp parallel for num_threads(orc_threads) schedule(static)
    for (int x = 0; x < lx; ++x)
        for (int p = 0; p < Q; ++p)
            for (int y = 0; y < ly; ++y) {
                const int sx = wrap((long)x - c[DIM * p], lx);
                const int sy = wrap((long)y - c[DIM * p + 1], ly);
                dst[at(p, x, y, lx, ly)] = src[at(p, sx, sy, lx, ly)];
            }
}

/* Collide every site in place. */
void orc_collide(int lx, int ly, const double *xi, const double *w, double tau, double *f)
{
#pragma omp parallel for num_threads(orc_threads) schedule(static)
    for (int x = 0; x < lx; ++x)
        for (int y = 0; y < ly; ++y) {
            double site[Q];
            for (int p = 0; p < Q; ++p) site[p] = f[at(p, x, y, lx, ly)];
            orc_collide_site(xi, w, tau, site);
            for (int p = 0; p < Q; ++p) f[at(p, x, y, lx, ly)] = site[p];
        }
}

/* nsteps x (propagate; collide). The result is left in f; tmp is a second
 * buffer of the same size. */
void orc_run(int lx, int ly, const int64_t *c, const double *xi, const double *w, double tau,
             int nsteps, double *f, double *tmp)
{
    const size_t n = (size_t)Q * lx * ly;
    for (int s = 0; s < nsteps; ++s) {
        orc_propagate(lx, ly, c, f, tmp);
        orc_collide(lx, ly, xi, w, tau, tmp);
        memcpy(f, tmp, n * sizeof(double));
    }
}

/* Macroscopic fields of every site. */
void orc_moments(int lx, int ly, const double *xi, const double *f, double *rho, double *ux,
                 double *uy, double *T)
{
    double site[Q];
    for (int x = 0; x < lx; ++x)
        for (int y = 0; y < ly; ++y) {
            const size_t s = (size_t)x * ly + y;
            for (int p = 0; p < Q; ++p) site[p] = f[at(p, x, y, lx, ly)];
            orc_moments_site(site, xi, &rho[s], &ux[s], &uy[s], &T[s]);
        }
}

/* Lattice totals: out = {mass, x-momentum, y-momentum, energy = 1/2 sum f xi.xi}. */
void orc_audit(int lx, int ly, const double *xi, const double *f, double *out)
{
    double m = 0.0, px = 0.0, py = 0.0, e = 0.0;
    for (int p = 0; p < Q; ++p) {
        const double x = xi[DIM * p], y = xi[DIM * p + 1];
        for (int xx = 0; xx < lx; ++xx)
            for (int yy = 0; yy < ly; ++yy) {
                const double v = f[at(p, xx, yy, lx, ly)];
                m += v;
                px += v * x;
                py += v * y;
                e += 0.5 * v * (x * x + y * y);
            }
    }
    out[0] = m;
    out[1] = px;
    out[2] = py;
    out[3] = e;
}

/* ---- Body force and walls ----------------------------------------------
 *
 * The paper's production runs (Section 3) follow a Rayleigh-Taylor system:
 * a fluid under gravity between a bottom and a top wall, the "Global"
 * timings of Section 5 including the kernels that apply them. The paper
 * defines neither, so these are the readings taken:
 *
 * Force (acceleration g per time step, thermal units): the equilibrium of
 * the collide is taken at a shifted velocity and temperature,
 *   u_s = u + tau g,  T_s = T + tau (1 - tau) |g|^2 / 2,
 *   f_i <- f_i - (f_i - f_eq_i(rho, u_s, T_s)) / tau.
 * The velocity shift is Shan and Chen's (Phys. Rev. E 47, 1815, 1993); the
 * temperature shift is fixed by energy: with the equilibrium's exact
 * moments, one step changes rho by 0, rho u by rho g and the energy
 * (1/2) sum f xi^2 by rho (u.g + |g|^2 / 2), the work of the force.
 *
 * Walls: diffuse reflection (Ansumali and Karlin, Phys. Rev. E 66, 026311,
 * 2002) on the planes y = -1/2 (bottom, temperature t_bottom) and
 * y = LY - 1/2 (top, t_top), at rest; x stays periodic. In the pull
 * propagate, a population whose source row y - c_y lies beyond a wall is
 * emitted by that wall: f_eq_p(rho_w(x_s), 0, T_w) with x_s = x - c_x the
 * source column. rho_w of a column makes the wall emit from it exactly the
 * mass that left the fluid towards the wall from that column in the same
 * propagate: the populations with c_y < 0 (bottom) in rows y < -c_y, or
 * c_y > 0 (top) in rows y >= LY - c_y. With K_w = sum over the populations
 * moving away from the wall of |c_y| f_eq_p(1, 0, T_w) (each is emitted
 * into |c_y| rows), rho_w = (outgoing mass of the column) / K_w. Total mass
 * is conserved exactly.
 */

/* Forced BGK collision of one site, in place. */
void orc_collide_site_force(const double *xi, const double *w, double tau, double gx, double gy, double *f)
{
    double rho, ux, uy, T, feq[Q];
    orc_moments_site(f, xi, &rho, &ux, &uy, &T);
    const double us_x = ux + tau * gx;
    const double us_y = uy + tau * gy;
    const double Ts = T + tau * (1.0 - tau) * (gx * gx + gy * gy) / 2.0;
    orc_feq_site(xi, w, rho, us_x, us_y, Ts, feq);
    for (int i = 0; i < Q; ++i) f[i] = f[i] - (f[i] - feq[i]) / tau;
}

/* Forced collide of every site in place. */
void orc_collide_force(int lx, int ly, const double *xi, const double *w, double tau, double gx, double gy,
                       double *f)
{
#pragma omp parallel for num_threads(orc_threads) schedule(static)
    for (int x = 0; x < lx; ++x)
        for (int y = 0; y < ly; ++y) {
            double site[Q];
            for (int p = 0; p < Q; ++p) site[p] = f[at(p, x, y, lx, ly)];
            orc_collide_site_force(xi, w, tau, gx, gy, site);
            for (int p = 0; p < Q; ++p) f[at(p, x, y, lx, ly)] = site[p];
        }
}

/* Wall densities rho_w[x] of one wall (bottom: side = 0, top: side = 1) from
 * the state src before propagation. */
static void wall_density(int lx, int ly, const int64_t *c, const double *xi, const double *w, int side,
                         double t_wall, const double *src, double *rho_w)
{
    double unit[Q];
    orc_feq_site(xi, w, 1.0, 0.0, 0.0, t_wall, unit);
    double K = 0.0;
    for (int p = 0; p < Q; ++p) {
        const long cy = (long)c[DIM * p + 1];
        if (side == 0 && cy > 0) K += (double)cy * unit[p];
        if (side == 1 && cy < 0) K += (double)(-cy) * unit[p];
    }
    for (int x = 0; x < lx; ++x) {
        double out = 0.0;
        for (int p = 0; p < Q; ++p) {
            const long cy = (long)c[DIM * p + 1];
            for (int y = 0; y < ly; ++y) {
                const int leaves = side == 0 ? (cy < 0 && y + cy < 0) : (cy > 0 && y + cy >= ly);
                if (leaves) out += src[at(p, x, y, lx, ly)];
            }
        }
        rho_w[x] = out / K;
    }
}

/* Pull propagate with diffuse walls at y = -1/2 and y = LY - 1/2, periodic
 * in x. rho_w is scratch of 2 * lx doubles. */
void orc_propagate_walls(int lx, int ly, const int64_t *c, const double *xi, const double *w, double t_bottom,
                         double t_top, const double *src, double *dst, double *rho_w)
{
    double *rho_b = rho_w, *rho_t = rho_w + lx;
    wall_density(lx, ly, c, xi, w, 0, t_bottom, src, rho_b);
    wall_density(lx, ly, c, xi, w, 1, t_top, src, rho_t);
#pragma omp parallel for num_threads(orc_threads) schedule(static)
    for (int x = 0; x < lx; ++x)
        for (int p = 0; p < Q; ++p)
            for (int y = 0; y < ly; ++y) {
                const int sx = wrap((long)x - c[DIM * p], lx);
                const long sy = (long)y - c[DIM * p + 1];
                double v;
                if (sy < 0 || sy >= ly) {
                    double feq[Q];
                    if (sy < 0) orc_feq_site(xi, w, rho_b[sx], 0.0, 0.0, t_bottom, feq);
                    else orc_feq_site(xi, w, rho_t[sx], 0.0, 0.0, t_top, feq);
                    v = feq[p];
                } else {
                    v = src[at(p, sx, (int)sy, lx, ly)];
                }
                dst[at(p, x, y, lx, ly)] = v;
            }
}

/* nsteps x (propagate; collide) with a body force g and, if walls != 0,
 * diffuse walls at the bottom and top. tmp is a second buffer of the size of
 * f, rho_w scratch of 2 * lx doubles. With g = 0 and walls = 0 this is
 * orc_run. */
void orc_run_bc(int lx, int ly, const int64_t *c, const double *xi, const double *w, double tau, double gx,
                double gy, int walls, double t_bottom, double t_top, int nsteps, double *f, double *tmp,
                double *rho_w)
{
    const size_t n = (size_t)Q * lx * ly;
    for (int s = 0; s < nsteps; ++s) {
        if (walls) orc_propagate_walls(lx, ly, c, xi, w, t_bottom, t_top, f, tmp, rho_w);
        else orc_propagate(lx, ly, c, f, tmp);
        orc_collide_force(lx, ly, xi, w, tau, gx, gy, tmp);
        memcpy(f, tmp, n * sizeof(double));
    }
}
