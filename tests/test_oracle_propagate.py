"""Pins of the oracle's propagate (Section 3 and Listing 1: every population
moves along its hop; a pure copy, no arithmetic)."""
import math

import numpy as np
import pytest

from oracle import lbm
from paper_1804_01918_amd import inputs


@pytest.fixture
def rand_f():
    def make(lx, ly, seed=0):
        return inputs.perturbation((37, lx, ly), seed)
    return make


@pytest.mark.parametrize("lx,ly", [(8, 8), (5, 7), (1, 1), (2, 9), (16, 3)])
def test_matches_numpy_roll(consts, rand_f, lx, ly):
    """Pull from x - c_p == shift the whole plane by +c_p (np.roll), bit-exact."""
    f = rand_f(lx, ly)
    g = lbm.propagate(f)
    for p, (cx, cy) in enumerate(consts["c"]):
        assert np.array_equal(g[p], np.roll(f[p], (int(cx), int(cy)), axis=(0, 1)))


@pytest.mark.parametrize("lx,ly", [(8, 8), (6, 4), (3, 5)])
def test_permutation_and_period(rand_f, lx, ly):
    f = rand_f(lx, ly, seed=3)
    g = f
    period = lx * ly // math.gcd(lx, ly)
    for k in range(period):
        g = lbm.propagate(g)
        assert np.array_equal(np.sort(g, axis=None), np.sort(f, axis=None))
        if k < period - 1 and min(lx, ly) > 3:
            assert not np.array_equal(g, f)
    assert np.array_equal(g, f)


def test_inverse_gather_restores(consts, rand_f):
    f = rand_f(9, 11, seed=5)
    g = lbm.propagate(f)
    opp = consts["opposite"]
    back = lbm.propagate(g[opp])[opp]
    assert np.array_equal(back, f)


def test_centre_of_mass_moves_with_hops(consts):
    """Sign convention: a population with hop c_p arrives at x + c_p. With a
    localised bump drifting in +x, the mass centroid moves by sum f c / sum f."""
    lx = ly = 32
    x = np.arange(lx)[:, None]
    y = np.arange(ly)[None, :]
    rho = 1 + 0.5 * np.exp(-((x - 16) ** 2 + (y - 16) ** 2) / 8.0)
    ux = np.full((lx, ly), 0.08)
    uy = np.full((lx, ly), -0.03)
    ones = np.ones((lx, ly))
    # Subtract the uniform background (itself invariant under propagate) so
    # that only the localised bump carries mass; it stays far from the edges.
    h = lbm.init(rho, ux, uy, ones) - lbm.init(ones, ux, uy, ones)
    c = consts["c"]
    M = h.sum()
    X = np.arange(lx)[None, :, None]
    Y = np.arange(ly)[None, None, :]
    cen = lambda a: np.array([(a * X).sum(), (a * Y).sum()]) / M
    expected = np.array([(h.sum(axis=(1, 2)) * c[:, 0]).sum(), (h.sum(axis=(1, 2)) * c[:, 1]).sum()]) / M
    assert expected[0] > 0 and expected[1] < 0
    g = lbm.propagate(h)
    assert abs(g.sum() - M) < 1e-12
    assert np.allclose(cen(g) - cen(h), expected, rtol=0, atol=1e-10)


@pytest.mark.parametrize("lx,ly,n", [(16, 16, 1), (16, 20, 2), (9, 7, 3)])
def test_run_window_matches_periodic_run(lx, ly, n):
    """The dependency-window evaluation equals the full periodic run bit for
    bit, including sites whose windows wrap around the edges."""
    fields = inputs.random_equilibrium(lx, ly, seed=6, amp=0.03)
    full = lbm.run(lbm.init(*fields), 0.8, n)
    sites = [(0, 0), (lx - 1, ly - 1), (lx // 2, 1), (3, ly - 2), (lx - 2, ly // 2)]
    got = lbm.run_window(fields, sites, n, 0.8)
    for k, (x, y) in enumerate(sites):
        assert np.array_equal(got[k], full[:, x, y])


def test_threaded_oracle_is_bit_identical_to_one_thread():
    """The all-core build of the oracle (column loops on several threads)
    gives the one-thread result bit for bit: init, propagate and collide are
    per site."""
    from oracle import lbm
    from paper_1804_01918_amd import inputs
    fields = inputs.random_equilibrium(45, 38, seed=4)
    try:
        lbm.set_threads(1)
        one = lbm.run(lbm.init(*fields), 0.7, 3)
        lbm.set_threads(4)
        assert lbm.get_threads() == 4
        many = lbm.run(lbm.init(*fields), 0.7, 3)
    finally:
        lbm.set_threads(1)
    assert np.array_equal(one.view(np.uint64), many.view(np.uint64))
