"""Pins of the oracle's equilibrium (reading of Section 3: fourth-order
Hermite expansion of the Maxwellian; the paper states the model enforces
p = rho T).

Independent route: moments of the continuous Maxwellian of density rho,
mean u and covariance T*I, computed by Gauss-Hermite quadrature in numpy.
"""
import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss

from oracle import lbm

STATES = [
    (1.0, 0.0, 0.0, 1.0),
    (1.03, 0.07, -0.02, 0.96),
    (0.91, -0.1, 0.05, 1.1),
    (1.1, 0.02, 0.09, 0.9),
]


def _maxwellian_moment(rho, ux, uy, T, a, b, n=16):
    z, wz = hermegauss(n)
    wz = wz / np.sqrt(2 * np.pi)
    X = ux + np.sqrt(T) * z[:, None]
    Y = uy + np.sqrt(T) * z[None, :]
    return rho * (np.outer(wz, wz) * X ** a * Y ** b).sum()


@pytest.mark.parametrize("state", STATES)
def test_moments_up_to_order_4_match_maxwellian(consts, state):
    rho, ux, uy, T = state
    f = lbm.feq_site(rho, ux, uy, T)
    xi = consts["xi"]
    for order in range(5):
        for a in range(order + 1):
            b = order - a
            got = (f * xi[:, 0] ** a * xi[:, 1] ** b).sum()
            exact = _maxwellian_moment(rho, ux, uy, T, a, b)
            assert abs(got - exact) <= 2e-14 * max(1.0, abs(exact)), (a, b, got, exact)


@pytest.mark.parametrize("state", STATES)
def test_perfect_gas_pressure(consts, state):
    """Pressure tensor sum f (xi-u)(xi-u) = rho T I, i.e. p = rho T."""
    rho, ux, uy, T = state
    f = lbm.feq_site(rho, ux, uy, T)
    d = consts["xi"] - np.array([ux, uy])
    P = np.einsum("i,ia,ib->ab", f, d, d)
    assert np.allclose(P, rho * T * np.eye(2), rtol=0, atol=1e-14)


@pytest.mark.parametrize("state", STATES)
def test_moments_recovered(state):
    rho, ux, uy, T = state
    got = lbm.moments_site(lbm.feq_site(rho, ux, uy, T))
    assert np.allclose(got, state, rtol=0, atol=1e-14)


def test_rest_state_is_weights(consts):
    assert np.allclose(lbm.feq_site(1.0, 0.0, 0.0, 1.0), consts["w"], rtol=1e-15, atol=0)


def test_fifth_order_not_matched(consts):
    """Truncation after fourth order: the fifth moment differs from the Maxwellian's."""
    rho, ux, uy, T = 1.0, 0.1, 0.0, 1.05
    f = lbm.feq_site(rho, ux, uy, T)
    got = (f * consts["xi"][:, 0] ** 5).sum()
    exact = _maxwellian_moment(rho, ux, uy, T, 5, 0)
    assert abs(got - exact) > 1e-6
