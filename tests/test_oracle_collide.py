"""Pins of the oracle's collide (Section 3: collide mixes the populations of
a site; reading: single-relaxation-time BGK towards the equilibrium)."""
import numpy as np
import pytest

from oracle import lbm
from paper_1804_01918_amd import inputs


def _noneq(consts, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    rho, ux, uy, T = 1 + 0.05 * rng.standard_normal(), *(0.05 * rng.standard_normal(2)), 1 + 0.05 * rng.standard_normal()
    f = lbm.feq_site(rho, ux, uy, T)
    return f + amp * consts["w"] * inputs.perturbation(37, seed + 1000)


@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 1.0), (1.05, 0.08, -0.03, 0.93), (0.9, -0.1, 0.1, 1.1)])
@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 2.5])
def test_equilibrium_is_fixed_point(consts, state, tau):
    f = lbm.feq_site(*state)
    g = lbm.collide_site(f, tau)
    assert np.max(np.abs(g - f) / consts["w"]) < 5e-15


@pytest.mark.parametrize("seed", range(6))
def test_conservation_per_site(consts, seed):
    xi = consts["xi"]
    f = _noneq(consts, seed)
    g = lbm.collide_site(f, 0.8)
    for phi in (np.ones(37), xi[:, 0], xi[:, 1], (xi ** 2).sum(1)):
        assert abs((g * phi).sum() - (f * phi).sum()) < 2e-15 * np.abs(f * phi).sum()


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.7])
def test_shear_stress_relaxes_by_one_minus_inverse_tau(consts, tau):
    """The non-equilibrium part of the off-diagonal stress sum f xi_x xi_y
    (equilibrium value rho ux uy) is multiplied by (1 - 1/tau) per collide."""
    xi = consts["xi"]
    f = _noneq(consts, 3, amp=1e-2)
    rho, ux, uy, T = lbm.moments_site(f)
    pi_neq = (f * xi[:, 0] * xi[:, 1]).sum() - rho * ux * uy
    g = lbm.collide_site(f, tau)
    pi_neq2 = (g * xi[:, 0] * xi[:, 1]).sum() - rho * ux * uy
    assert abs(pi_neq2 - (1 - 1 / tau) * pi_neq) < 1e-15 + 1e-12 * abs(pi_neq)


def test_tau_one_gives_equilibrium(consts):
    f = _noneq(consts, 9, amp=1e-2)
    g = lbm.collide_site(f, 1.0)
    assert np.max(np.abs(g - lbm.feq_site(*lbm.moments_site(f))) / consts["w"]) < 1e-14
