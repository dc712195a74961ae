"""Pins of the oracle's lattice audit and of the learning-rate schedule.

* The audit (orc_audit) sums mass, momentum and energy 1/2 sum f |xi|^2 over
  the lattice. It is pinned three ways that do not reuse its own formula:
  - closed form: a uniform equilibrium (rho0, u0, T0) on N sites has
    M = N rho0, P = N rho0 u0 and E = N rho0 (|u0|^2 / 2 + T0) (the
    equilibrium's first and second moments, with D = 2 degrees of freedom,
    Section 3's p = rho T);
  - the per-site macroscopic fields of orc_moments summed over the lattice:
    sum rho, sum rho u, sum rho (|u|^2 + 2 T) / 2;
  - conservation: collide conserves mass, momentum and energy and propagate
    only permutes values, so the totals stay constant over 100 steps.
  A dropped factor 1/2, lattice hops c used in place of thermal velocities
  xi = r c, or a missing population fails at least one of them.
* cosine_lr: lr0 (1 + cos(pi s / S)) / 2 is lr0 at s = 0, lr0 / 2 at S / 2,
  0 at S, and symmetric about S / 2 in the sense lr(s) + lr(S - s) = lr0.
"""
import math

import numpy as np
import pytest

from oracle import lbm
from oracle import surrogate as S
from paper_1804_01918_amd import inputs


@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 1.0), (1.07, 0.04, -0.09, 0.93), (0.95, -0.1, 0.02, 1.1)])
def test_audit_closed_form_uniform_equilibrium(state):
    rho0, ux0, uy0, T0 = state
    lx, ly = 5, 7
    n = lx * ly
    fields = [np.full((lx, ly), v) for v in state]
    f = lbm.init(*fields)
    got = lbm.audit(f)
    want = np.array([n * rho0, n * rho0 * ux0, n * rho0 * uy0, n * rho0 * (0.5 * (ux0 ** 2 + uy0 ** 2) + T0)])
    # recursive summation of 37 N terms: error <= 37 N 2^-53 times the sum
    # of the magnitudes (about M for mass and momentum, E for energy)
    scale = np.array([want[0], want[0], want[0], want[3]])
    assert np.all(np.abs(got - want) <= 37 * n * 2.0 ** -53 * scale), (got, want)


@pytest.mark.parametrize("kind", ["random_equilibrium", "shear_wave", "rayleigh_taylor"])
def test_audit_equals_sum_of_site_moments(consts, kind):
    lx, ly = 12, 20
    f = lbm.init(*inputs.make_state(kind, lx, ly, seed=3))
    # a non-equilibrium state: one step plus a perturbation of every population
    f = lbm.run(f, 0.8, 1) + 1e-3 * consts["w"][:, None, None] * inputs.perturbation(f.shape, 5)
    rho, ux, uy, T = lbm.moments(f)
    want = np.array([rho.sum(), (rho * ux).sum(), (rho * uy).sum(),
                     (0.5 * rho * (ux * ux + uy * uy + 2.0 * T)).sum()])
    got = lbm.audit(f)
    scale = rho.sum()
    assert np.all(np.abs(got - want) <= 1e-14 * scale), (got - want)


@pytest.mark.parametrize("kind", ["random_equilibrium", "rayleigh_taylor"])
def test_audit_constant_over_steps(kind):
    lx, ly = 16, 24
    f = lbm.init(*inputs.make_state(kind, lx, ly, seed=1))
    a0 = lbm.audit(f)
    f = lbm.run(f, 0.8, 100)
    a1 = lbm.audit(f)
    assert np.all(np.abs(a1 - a0) <= 1e-13 * a0[0]), (a1 - a0)


def test_audit_sees_every_population(consts):
    """Adding delta to one population p at one site moves the totals by
    (delta, delta xi_p, delta |xi_p|^2 / 2)."""
    xi = consts["xi"]
    f = lbm.init(*inputs.random_equilibrium(6, 6, seed=2))
    a0 = lbm.audit(f)
    for p in (0, 11, 18, 29, 36):
        g = f.copy()
        g[p, 4, 1] += 0.25
        d = lbm.audit(g) - a0
        want = 0.25 * np.array([1.0, xi[p, 0], xi[p, 1], 0.5 * (xi[p] ** 2).sum()])
        assert np.all(np.abs(d - want) < 1e-13), (p, d, want)


@pytest.mark.parametrize("lr0,total", [(3e-3, 1000), (1.0, 7), (0.5, 39040)])
def test_cosine_lr_closed_form(lr0, total):
    assert S.cosine_lr(lr0, 0, total) == lr0
    assert abs(S.cosine_lr(lr0, total / 2, total) - lr0 / 2) <= 1e-16 * lr0
    assert abs(S.cosine_lr(lr0, total, total)) <= 1e-16 * lr0
    for s in range(0, total + 1, max(1, total // 13)):
        assert abs(S.cosine_lr(lr0, s, total) + S.cosine_lr(lr0, total - s, total) - lr0) <= 1e-15 * lr0
        if s > 0:
            assert S.cosine_lr(lr0, s, total) <= S.cosine_lr(lr0, s - 1, total)
    # a quarter of the way: lr0 (1 + cos(pi/4)) / 2
    assert abs(S.cosine_lr(lr0, total / 4, total) - lr0 * (2 + math.sqrt(2)) / 4) <= 1e-15 * lr0
