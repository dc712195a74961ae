// Site-local collide of the D2Q37 model (paper, Section 3: moments rho, u,
// T; the thermal equilibrium of the model, which enforces p = rho T; then
// relaxation; about 6600 flops per site in the paper's code).
//
// Equilibrium: fourth-order Hermite expansion of the Maxwellian in thermal
// units xi = R c. For population i with x = xi_i . u and X2 = |xi_i|^2 it is
// a quartic in x whose coefficients depend only on the shell of i:
//   f_eq_i = w_i rho (A0 + A1 x + A2 x^2 + x^3/6 + x^4/24)
//   A0 = 1 - u2/2 + t (X2-2)/2 + [3 u2^2 + 6 t u2 (4-X2) + 3 t^2 (X2^2 - 8 X2 + 8)]/24
//   A1 = 1 - u2/2 + t (X2-4)/2
//   A2 = 1/2 - u2/4 + t (X2-6)/4,         t = T - 1, u2 = u.u.
// Opposite populations share X2 and have opposite x, so each pair needs one
// even and one odd Horner chain. BGK relaxation with omega = 1/tau is folded
// into the shell coefficients: f'_i = (1 - omega) f_i + omega f_eq_i. This
// costs about 400 flops per site instead of the paper's 6600.
//
// Shifted form (populations stored as g = f - w with rho0 = 1): since
// sum w = 1, sum w xi = 0 and sum w xi^2 = 2,
//   rho - 1 = sum g,  rho u = sum g xi,  2 rho (T - 1) = sum g (xi^2 - 2) - rho u2,
//   g_eq_i = w_i [(rho - 1) + rho (P_i - 1)]  with P_i the bracket above.
#pragma once

#include "lb_layout.hpp"

namespace d2q37 {

// Explicit fused multiply-add. The library is compiled without automatic
// contraction, so every kernel that shares these functions rounds the same.
__device__ inline double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Product with a model constant k. In FP32 the constant is carried as a
// pair hi + lo (hi = k rounded to FP32, lo = the FP32 rounding of the rest),
// so the product is as accurate as with a ~48-bit constant. A single rounded
// constant would bias the moments of the equilibrium by ~3e-8 relative (for
// example its momentum by rho u (1 + delta)), and that bias accumulates
// coherently over the steps.
__device__ inline double mulk(double a, double k) { return a * k; }
__device__ inline float mulk(float a, double k)
{
    const float hi = (float)k;
    const float lo = (float)(k - (double)hi);
    return __builtin_fmaf(a, hi, a * lo);
}

// ---- compensated FP32 summation ------------------------------------------
// Knuth's TwoSum: a + b = s + e exactly, for any ordering of |a|, |b|.
__device__ inline void two_sum(float a, float b, float& s, float& e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Cascaded TwoSum with the rounding errors accumulated apart (Ogita, Rump
// and Oishi, "Accurate sum and dot product", SIAM J. Sci. Comput. 26, 2005:
// algorithms Sum2 / Dot2). Result as if summed in twice the precision.
struct CompSum {
    float s = 0.0f, c = 0.0f;
    __device__ void add(float x)
    {
        float e;
        two_sum(s, x, s, e);
        c += e;
    }
    // Adds k * (v + ev), where ev is the known error of v; the product's own
    // rounding error is recovered with an FMA (TwoProduct).
    __device__ void add_scaled(float k, float v, float ev)
    {
        const float p = k * v;
        const float pe = __builtin_fmaf(k, v, -p);
        add(p);
        c += fma_(k, ev, pe);
    }
    __device__ float value() const { return s + c; }
};

// Moments of a site in lattice units: sum v, sum cx v, sum cy v, sum |c|^2 v.
template <typename C>
struct RawMoments {
    C m0, jx, jy, e;
};

template <typename C>
__device__ inline RawMoments<C> raw_moments_plain(const C (&v)[Q])
{
    C m0 = v[REST], e = C(0), jx = C(0), jy = C(0);
#pragma unroll
    for (int i = 0; i < NPAIR; ++i) {
        const int o = Q - 1 - i;
        const C ps = v[i] + v[o];
        const C pd = v[i] - v[o];
        m0 += ps;
        e = fma_(C(c2_of(i)), ps, e);
        if (CX[i] != 0) jx = fma_(C(CX[i]), pd, jx);
        if (CY[i] != 0) jy = fma_(C(CY[i]), pd, jy);
    }
    return {m0, jx, jy, e};
}

__device__ inline RawMoments<float> raw_moments_compensated(const float (&v)[Q])
{
    CompSum m0, jx, jy, e;
    m0.s = v[REST];
#pragma unroll
    for (int i = 0; i < NPAIR; ++i) {
        const int o = Q - 1 - i;
        float ps, eps, pd, epd;
        two_sum(v[i], v[o], ps, eps);
        two_sum(v[i], -v[o], pd, epd);
        m0.add(ps);
        m0.c += eps;
        e.add_scaled(float(c2_of(i)), ps, eps);
        if (CX[i] != 0) jx.add_scaled(float(CX[i]), pd, epd);
        if (CY[i] != 0) jy.add_scaled(float(CY[i]), pd, epd);
    }
    return {m0.value(), jx.value(), jy.value(), e.value()};
}

// Macroscopic state entering the equilibrium.
template <typename C>
struct Macro {
    C drho;  // rho - 1 (shifted) or rho (plain): the density term of B0
    C rho;
    C Ux, Uy;  // R * u: x_i = cx_i Ux + cy_i Uy equals xi_i . u
    C u2;      // |u|^2 in thermal units
    C t;       // T - 1
};

template <typename C, bool SHIFTED>
__device__ inline Macro<C> macro_from_raw(const RawMoments<C>& m)
{
    Macro<C> s;
    if constexpr (SHIFTED) {
        s.drho = m.m0;
        s.rho = C(1) + m.m0;
    } else {
        s.drho = m.m0;
        s.rho = m.m0;
    }
    const C inv_rho = C(1) / s.rho;
    s.Ux = mulk(m.jx, R2) * inv_rho;
    s.Uy = mulk(m.jy, R2) * inv_rho;
    s.u2 = mulk(s.Ux * s.Ux + s.Uy * s.Uy, THETA);
    if constexpr (SHIFTED)
        s.t = (mulk(m.e, R2) - C(2) * m.m0 - s.rho * s.u2) * (C(0.5) * inv_rho);
    else
        s.t = C(0.5) * (mulk(m.e, R2) * inv_rho - s.u2) - C(1);
    return s;
}

// Relaxation towards the equilibrium, shell by shell:
//   emit(i, omw * v_i + omega * equilibrium_i)   (plain: f_eq; shifted: g_eq)
// for every population. omega = 1, omw = 0 gives the equilibrium itself.
// A shell's coefficients are formed just before its populations are emitted,
// which keeps few of them live at once.
template <typename C, bool SHIFTED, class Emit>
__device__ inline void relax_emit(const C (&v)[Q], const Macro<C>& s, C omega, C omw, Emit&& emit)
{
    const C kr = omega * s.rho;
    const C u2 = s.u2, t = s.t;
#pragma unroll
    for (int h = 0; h < NSHELL; ++h) {
        const C X2 = C(R2 * SHELL_C2[h]);
        const C q4 = C(R2 * SHELL_C2[h] * (R2 * SHELL_C2[h] - 8.0) + 8.0);  // X2^2 - 8 X2 + 8
        const C K = mulk(kr, WSH[h]);
        // A0 - 1
        const C a0m1 = -C(0.5) * u2 + C(0.5) * t * (X2 - C(2))
                       + (C(3) * u2 * u2 + C(6) * t * u2 * (C(4) - X2) + C(3) * t * t * q4) * C(1.0 / 24.0);
        C B0;
        if constexpr (SHIFTED)
            B0 = mulk(omega * s.drho, WSH[h]) + K * a0m1;
        else
            B0 = K * (C(1) + a0m1);
        if (h == 0) {
            emit(REST, fma_(omw, v[REST], B0));
            continue;
        }
        const C B1 = K * (C(1) - C(0.5) * u2 + C(0.5) * t * (X2 - C(4)));
        const C B2 = K * (C(0.5) - C(0.25) * u2 + C(0.25) * t * (X2 - C(6)));
        const C B3 = K * C(1.0 / 6.0);
        const C B4 = K * C(1.0 / 24.0);
#pragma unroll
        for (int i = 0; i < NPAIR; ++i) {
            if (shell_of_c2(c2_of(i)) != h) continue;
            const int o = Q - 1 - i;
            C x;
            if (CX[i] == 0) x = C(CY[i]) * s.Uy;
            else if (CY[i] == 0) x = C(CX[i]) * s.Ux;
            else x = fma_(C(CX[i]), s.Ux, C(CY[i]) * s.Uy);
            const C x2 = x * x;
            const C ev = fma_(x2, fma_(x2, B4, B2), B0);
            const C od = x * fma_(x2, B3, B1);
            emit(i, fma_(omw, v[i], ev + od));
            emit(o, fma_(omw, v[o], ev - od));
        }
    }
}

// Body force g (acceleration per step, thermal units): the collide relaxes
// towards the equilibrium at the shifted velocity u + tau g and temperature
// T + tau (1 - tau) |g|^2 / 2 (a velocity shift of the equilibrium, with the
// temperature shift that makes the energy gain exactly the work of the
// force). Per step a site keeps its mass, gains rho g of momentum and
// rho (u.g + |g|^2 / 2) of energy. Held as the shifts of (Ux, Uy) = R u and
// of t = T - 1; zero shifts leave every rounding of the plain collide as is.
template <typename C>
struct Force {
    C dUx, dUy;  // R tau g
    C dt;        // tau (1 - tau) |g|^2 / 2
};

template <typename C>
__device__ inline void apply_force(Macro<C>& s, const Force<C>& f)
{
    s.Ux += f.dUx;
    s.Uy += f.dUy;
    s.u2 = mulk(s.Ux * s.Ux + s.Uy * s.Uy, THETA);
    s.t += f.dt;
}

// BGK collide of one site held in registers, with a body force if FORCE;
// emit(p, value) receives the post-collision populations.
template <class P, bool COMP, bool FORCE, class Emit>
__device__ inline void collide_site_f(const typename P::C (&v)[Q], typename P::C omega,
                                      const Force<typename P::C>& force, Emit&& emit)
{
    using C = typename P::C;
    RawMoments<C> m;
    if constexpr (P::shifted && COMP && sizeof(C) == 4)
        m = raw_moments_compensated(v);
    else
        m = raw_moments_plain(v);
    Macro<C> s = macro_from_raw<C, P::shifted>(m);
    if constexpr (FORCE) apply_force(s, force);
    relax_emit<C, P::shifted>(v, s, omega, C(1) - omega, emit);
}

template <class P, bool COMP, class Emit>
__device__ inline void collide_site(const typename P::C (&v)[Q], typename P::C omega, Emit&& emit)
{
    collide_site_f<P, COMP, false>(v, omega, Force<typename P::C>{}, emit);
}

// Equilibrium (plain f_eq or shifted g_eq) from FP64 fields, in FP64.
template <bool SHIFTED, class Emit>
__device__ inline void equilibrium_f64(double rho, double ux, double uy, double T, Emit&& emit)
{
    Macro<double> s;
    s.rho = rho;
    s.drho = SHIFTED ? rho - 1.0 : rho;
    s.Ux = R * ux;
    s.Uy = R * uy;
    s.u2 = ux * ux + uy * uy;
    s.t = T - 1.0;
    double zero[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) zero[p] = 0.0;
    relax_emit<double, SHIFTED>(zero, s, 1.0, 0.0, emit);
}

}  // namespace d2q37
