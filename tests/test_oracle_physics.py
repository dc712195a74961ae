"""Whole-step pins of the oracle against kinetic theory, lattice symmetry
and an arbitrary-precision brute force built on a different route.

* Shear wave: the BGK model has kinematic viscosity nu = theta T (tau - 1/2)
  in lattice units (theta = 1/r^2 is the squared lattice sound speed at
  T = 1), so a sinusoidal shear mode decays as exp(-nu k^2 t).
* Sound wave: the perfect-gas equation of state p = rho T (Section 3) with
  two translational degrees of freedom gives an adiabatic exponent of 2, so
  a standing pressure wave oscillates at c_s k with c_s = sqrt(2 theta T).
* Symmetry: a 90 degree rotation or a mirror of the initial state commutes
  with the time step.
* Brute force: 40-digit mpmath run of the same step in which the equilibrium
  is assembled from one-dimensional probabilists' Hermite polynomials and
  Gaussian expectations (not the tensor formulas of the C oracle).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import lbm
from paper_1804_01918_amd import inputs


def _mode(field, k_axis_len, kind):
    y = np.arange(k_axis_len)
    basis = np.sin(2 * np.pi * y / k_axis_len) if kind == "sin" else np.cos(2 * np.pi * y / k_axis_len)
    return 2.0 * (field.mean(axis=0) * basis).mean()


@pytest.mark.parametrize("ly,tol", [(32, 1e-2), (64, 3e-3), (128, 1e-3)])
def test_shear_wave_decay(consts, ly, tol):
    lx, tau, U = 4, 0.8, 0.005
    rho, ux, uy, T = inputs.shear_wave(lx, ly, noise=0.0, u0=U)
    f = lbm.init(rho, ux, uy, T)
    ts, amps = [], []
    t = 0
    for t_next in range(50, 601, 50):
        f = lbm.run(f, tau, t_next - t)
        t = t_next
        _, vx, _, _ = lbm.moments(f)
        ts.append(t)
        amps.append(_mode(vx, ly, "sin"))
    slope = np.polyfit(ts, np.log(amps), 1)[0]
    k = 2 * np.pi / ly
    nu = consts["theta"] * 1.0 * (tau - 0.5)
    assert abs(-slope / (nu * k * k) - 1.0) < tol


def test_sound_speed_is_adiabatic(consts):
    lx, ly, tau, A = 4, 64, 0.8, 1e-3
    y = np.arange(ly)
    rho = np.broadcast_to(1 + A * np.cos(2 * np.pi * y / ly), (lx, ly)).copy()
    zero = np.zeros((lx, ly))
    f = lbm.init(rho, zero, zero, np.ones((lx, ly)))
    vals = []
    for _ in range(320):
        f = lbm.run(f, tau, 1)
        _, _, vy, _ = lbm.moments(f)
        vals.append(_mode(vy, ly, "sin"))
    vals = np.array(vals)
    t = np.arange(1, 321)
    idx = np.where(np.sign(vals[:-1]) != np.sign(vals[1:]))[0]
    zc = t[idx] + vals[idx] / (vals[idx] - vals[idx + 1])
    half_period = (zc[-1] - zc[0]) / (len(zc) - 1)
    c_meas = (np.pi / half_period) / (2 * np.pi / ly)
    c_adiabatic = math.sqrt(2.0 * consts["theta"])
    assert len(zc) >= 8
    assert abs(c_meas / c_adiabatic - 1.0) < 1e-2


def _rotate90(f, consts):
    """(x, y) -> (-y, x) on an L x L lattice; population c -> R c."""
    c = consts["c"]
    L = f.shape[1]
    index = {tuple(v): i for i, v in enumerate(c)}
    out = np.empty_like(f)
    xs, ys = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    for p, (cx, cy) in enumerate(c):
        q = index[(-int(cy), int(cx))]
        out[q, (-ys) % L, xs] = f[p]
    return out


def _mirror_x(f, consts):
    c = consts["c"]
    L = f.shape[1]
    index = {tuple(v): i for i, v in enumerate(c)}
    out = np.empty_like(f)
    for p, (cx, cy) in enumerate(c):
        q = index[(-int(cx), int(cy))]
        out[q] = f[p][(-np.arange(L)) % L, :]
    return out


@pytest.mark.parametrize("op", ["rot90", "mirror"])
def test_symmetry_commutes_with_step(consts, op):
    L = 16
    f0 = lbm.init(*inputs.random_equilibrium(L, L, seed=4, amp=0.03))
    f0 = f0 + 1e-3 * consts["w"][:, None, None] * inputs.perturbation(f0.shape, 11)
    tr = (lambda a: _rotate90(a, consts)) if op == "rot90" else (lambda a: _mirror_x(a, consts))
    a = tr(lbm.run(f0, 0.8, 6))
    b = lbm.run(tr(f0), 0.8, 6)
    assert np.max(np.abs(a - b) / consts["w"][:, None, None]) < 1e-13


# ---- arbitrary-precision brute force --------------------------------------

def _he(n, x):
    """Probabilists' Hermite polynomial He_n(x) by its three-term recurrence."""
    h0, h1 = mp.mpf(1), x
    if n == 0:
        return h0
    for m in range(1, n):
        h0, h1 = h1, x * h1 - m * h0
    return h1


def _he_coeffs(n):
    """Monomial coefficients of He_n (ascending powers)."""
    prev, cur = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    if n == 0:
        return prev
    for m in range(1, n):
        nxt = [mp.mpf(0)] + cur
        for j, v in enumerate(prev):
            nxt[j] -= m * v
        prev, cur = cur, nxt
    return cur


def _gauss_expect_he(n, u, T):
    """E[He_n(u + sqrt(T) Z)], Z standard normal, from binomial expansion and
    the Gaussian moments E[Z^m] = (m-1)!! (m even)."""
    s = mp.sqrt(T)
    total = mp.mpf(0)
    for k, a in enumerate(_he_coeffs(n)):
        for m in range(0, k + 1, 2):
            dfact = mp.mpf(1)
            for j in range(m - 1, 0, -2):
                dfact *= j
            total += a * mp.binomial(k, m) * u ** (k - m) * s ** m * dfact
    return total


def _feq_mp(xi, w, rho, ux, uy, T):
    bx = [_gauss_expect_he(n, ux, T) for n in range(5)]
    by = [_gauss_expect_he(n, uy, T) for n in range(5)]
    out = []
    for (x, y), wi in zip(xi, w):
        s = mp.mpf(0)
        for nx in range(5):
            for ny in range(5 - nx):
                s += bx[nx] * by[ny] * _he(nx, x) * _he(ny, y) / (mp.factorial(nx) * mp.factorial(ny))
        out.append(wi * rho * s)
    return out


def test_brute_force_mpmath_8x8(consts):
    mp.mp.dps = 40
    from oracle.lattice import solve_quadrature, velocities
    w_sh, theta, _ = solve_quadrature(50)
    mp.mp.dps = 40
    c = velocities()
    r = 1 / mp.sqrt(theta)
    xi_mp = [(r * int(cx), r * int(cy)) for cx, cy in c]
    w_mp = [w_sh[int(cx * cx + cy * cy)] for cx, cy in c]
    L, steps, tau = 8, 3, mp.mpf("0.8")
    f0 = lbm.init(*inputs.random_equilibrium(L, L, seed=2, amp=0.05))
    f0 = f0 + 1e-3 * consts["w"][:, None, None] * inputs.perturbation(f0.shape, 12)
    F = [[[mp.mpf(float(f0[p, x, y])) for y in range(L)] for x in range(L)] for p in range(37)]
    for _ in range(steps):
        G = [[[F[p][(x - int(c[p][0])) % L][(y - int(c[p][1])) % L] for y in range(L)] for x in range(L)]
             for p in range(37)]
        for x in range(L):
            for y in range(L):
                fs = [G[p][x][y] for p in range(37)]
                rho = mp.fsum(fs)
                jx = mp.fsum(fv * xv[0] for fv, xv in zip(fs, xi_mp))
                jy = mp.fsum(fv * xv[1] for fv, xv in zip(fs, xi_mp))
                e = mp.fsum(fv * (xv[0] ** 2 + xv[1] ** 2) for fv, xv in zip(fs, xi_mp))
                ux, uy = jx / rho, jy / rho
                T = (e / rho - ux * ux - uy * uy) / 2
                feq = _feq_mp(xi_mp, w_mp, rho, ux, uy, T)
                for p in range(37):
                    G[p][x][y] = fs[p] - (fs[p] - feq[p]) / tau
        F = G
    got = lbm.run(f0, 0.8, steps)
    exact = np.array([[[float(F[p][x][y]) for y in range(L)] for x in range(L)] for p in range(37)])
    # FP64 rounding of three steps, measured per population against its
    # weight (the scale of f_p); a wrong term in the equilibrium shows at 1e-4.
    assert np.max(np.abs(got - exact) / consts["w"][:, None, None]) < 3e-14
