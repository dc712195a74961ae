"""Pins of the oracle's velocity set and quadrature (model of Section 3).

The weights come from a Newton solve (oracle/lattice.py); they are checked
here against an independent route: tensor-product Gauss-Hermite quadrature
from numpy, which integrates polynomials against the unit Gaussian exactly
up to a known degree.
"""
import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss

from oracle.lattice import Q, solve_quadrature


def test_velocity_set(consts):
    c = consts["c"]
    assert c.shape == (Q, 2)
    c2 = (c * c).sum(1)
    counts = {int(s): int((c2 == s).sum()) for s in np.unique(c2)}
    assert counts == {0: 1, 1: 4, 2: 4, 4: 4, 5: 8, 8: 4, 9: 4, 10: 8}
    # "moving up to three lattice points away" (Section 3)
    assert np.abs(c).max() == 3
    assert len({tuple(v) for v in c}) == Q
    assert tuple(c[18]) == (0, 0)
    for i in range(Q):
        assert tuple(c[Q - 1 - i]) == tuple(-c[i])


def test_weights_positive_and_normalised(consts):
    w = consts["w"]
    assert (w > 0).all()
    assert abs(w.sum() - 1.0) < 1e-15
    _, _, res = solve_quadrature()
    assert res < 1e-40


def _gauss_hermite_2d(fun, n=12):
    z, wz = hermegauss(n)
    wz = wz / np.sqrt(2 * np.pi)
    X, Y = np.meshgrid(z, z, indexing="ij")
    W = np.outer(wz, wz)
    return (W * fun(X, Y)).sum()


def _lattice_sum(consts, fun):
    xi = consts["xi"]
    return (consts["w"] * fun(xi[:, 0], xi[:, 1])).sum()


@pytest.mark.parametrize("degree", range(0, 10))
def test_exact_up_to_degree_9(consts, degree):
    """sum_i w_i q(xi_i) equals the Gaussian integral of q for deg(q) <= 9."""
    rng = np.random.default_rng(100 + degree)
    for _ in range(5):
        coef = rng.standard_normal(degree + 1)

        def q(x, y, coef=coef):
            return sum(coef[a] * x ** a * y ** (degree - a) for a in range(degree + 1))

        exact = _gauss_hermite_2d(q)
        got = _lattice_sum(consts, q)
        scale = max(1.0, np.abs(coef).sum() * 3.0 ** degree)
        assert abs(got - exact) <= 1e-14 * scale, (degree, got, exact)


def test_not_exact_at_degree_10(consts):
    """The set is a degree-9 quadrature, not more: x^10 is not integrated."""
    exact = _gauss_hermite_2d(lambda x, y: x ** 10)   # 9!! = 945
    got = _lattice_sum(consts, lambda x, y: x ** 10)
    assert abs(exact - 945.0) < 1e-9
    assert abs(got / exact - 1.0) > 1e-2


def test_isotropy_random_directions(consts):
    """sum w (n.xi)^k is the same for every unit n, k = 2,4,6,8, and equals (k-1)!!."""
    xi, w = consts["xi"], consts["w"]
    rng = np.random.default_rng(7)
    for phi in rng.uniform(0, 2 * np.pi, 8):
        n = np.array([np.cos(phi), np.sin(phi)])
        proj = xi @ n
        for k, df in ((2, 1.0), (4, 3.0), (6, 15.0), (8, 105.0)):
            assert abs((w * proj ** k).sum() - df) < 1e-12 * df
