"""Pins of the oracle's body force and walls (the Rayleigh-Taylor setting of
the paper's Section 3: gravity, bottom and top walls) against closed forms,
conservation laws, symmetries and textbook flows.

Readings (the paper defines neither): the force shifts the equilibrium's
velocity by tau g and its temperature by tau (1 - tau) |g|^2 / 2; the walls
are diffuse reflectors at rest at y = -1/2 and y = LY - 1/2 whose emitted
mass per column equals the mass that left the fluid from that column.
Lattice units: y in sites, time in steps; g and u in thermal units, so an
acceleration g is g / r sites per step^2 and the kinematic viscosity is
theta T (tau - 1/2) sites^2 per step (theta = 1 / r^2)."""
import numpy as np
import pytest

from oracle import lbm
from paper_1804_01918_amd import inputs


def _uniform(lx, ly, rho=1.0, T=1.0):
    return (np.full((lx, ly), rho), np.zeros((lx, ly)), np.zeros((lx, ly)), np.full((lx, ly), T))


def _energy(f, xi):
    return 0.5 * np.einsum("p...,p->...", f, (xi ** 2).sum(axis=1))


def test_no_force_no_walls_is_the_plain_step():
    f0 = lbm.init(*inputs.random_equilibrium(9, 13, seed=3))
    a = lbm.run(f0, 0.8, 4)
    b = lbm.run_bc(f0, 0.8, 4, g=(0.0, 0.0), walls=False)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 2.5])
def test_forced_collide_adds_exactly_momentum_and_work(consts, tau):
    """Per site: mass unchanged, momentum + rho g, energy + rho (u.g + g^2/2)
    (the work of the force over one step), to FP64 rounding."""
    xi = consts["xi"]
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho, T = 1 + 0.05 * rng.standard_normal(), 1 + 0.05 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(2)
        g = 2e-3 * rng.standard_normal(2)
        f = lbm.feq_site(rho, u[0], u[1], T) * (1 + 1e-3 * rng.standard_normal(37))
        m0, j0, e0 = f.sum(), f @ xi, _energy(f, xi)
        ubar = j0 / m0
        out = lbm.collide_site_force(f, tau, g)
        assert abs(out.sum() - m0) <= 1e-15 * m0
        assert np.all(np.abs(out @ xi - (j0 + m0 * g)) <= 1e-15 * m0)
        de = m0 * (ubar @ g + 0.5 * g @ g)
        assert abs(_energy(out, xi) - (e0 + de)) <= 1e-14 * e0


def test_uniform_acceleration_closed_form(consts):
    """A uniform fluid at rest under a uniform force in a periodic box: after
    n steps every site has rho unchanged, velocity n g and the starting
    temperature (its energy grew by exactly rho n^2 g^2 / 2)."""
    lx, ly, tau, n = 6, 5, 0.8, 12
    g = np.array([3e-3, -2e-3])
    f = lbm.run_bc(lbm.init(*_uniform(lx, ly, 1.1, 0.95)), tau, n, g=g)
    rho, ux, uy, T = lbm.moments(f)
    assert np.allclose(rho, 1.1, rtol=0, atol=1e-14)
    assert np.allclose(ux, n * g[0], rtol=0, atol=1e-15)
    assert np.allclose(uy, n * g[1], rtol=0, atol=1e-15)
    assert np.allclose(T, 0.95, rtol=0, atol=1e-14)


def test_walls_keep_the_rest_state_at_their_temperature(consts):
    """Fluid at rest at the walls' temperature is a fixed point: the walls
    re-emit exactly the equilibrium they absorb."""
    f0 = lbm.init(*_uniform(4, 16, 1.0, 1.03))
    f = lbm.run_bc(f0, 0.8, 20, walls=True, t_bottom=1.03, t_top=1.03)
    w = consts["w"][:, None, None]
    assert np.max(np.abs(f - f0) / w) < 1e-13


@pytest.mark.parametrize("g", [(0.0, 0.0), (1e-3, -2e-3)])
def test_walls_conserve_mass(g):
    """Diffuse walls with different temperatures and a force: the lattice
    mass stays constant (each column's wall emits what left it)."""
    f0 = lbm.init(*inputs.random_equilibrium(12, 20, seed=2))
    m0 = lbm.audit(f0)[0]
    f = lbm.run_bc(f0, 0.8, 40, g=g, walls=True, t_bottom=1.05, t_top=0.95)
    assert abs(lbm.audit(f)[0] - m0) <= 1e-13 * m0


def test_walls_change_momentum_and_energy():
    """The walls are not conservative for momentum (they are at rest) nor
    for energy (they hold their temperature): a sheared, hot fluid between
    cold walls loses x-momentum and energy."""
    lx, ly = 4, 12
    rho, ux, uy, T = _uniform(lx, ly, 1.0, 1.05)
    ux = ux + 0.05
    f0 = lbm.init(rho, ux, uy, T)
    a0 = lbm.audit(f0)
    a = lbm.audit(lbm.run_bc(f0, 0.8, 30, walls=True, t_bottom=1.0, t_top=1.0))
    assert a[1] < 0.9 * a0[1]
    assert a[3] < a0[3]


def test_mirror_symmetry_of_walls_and_force(consts):
    """Mirroring y -> LY - 1 - y (c_y -> -c_y, g_y -> -g_y, bottom and top
    walls exchanged) commutes with the step."""
    c = consts["c"]
    mirror = [int(np.flatnonzero((c[:, 0] == cx) & (c[:, 1] == -cy))[0]) for cx, cy in c]
    f0 = lbm.init(*inputs.random_equilibrium(7, 15, seed=5))
    g = (1e-3, 2e-3)
    a = lbm.run_bc(f0, 0.8, 6, g=g, walls=True, t_bottom=1.04, t_top=0.97)
    m0 = f0[mirror][:, :, ::-1]
    b = lbm.run_bc(m0, 0.8, 6, g=(g[0], -g[1]), walls=True, t_bottom=0.97, t_top=1.04)
    w = consts["w"][:, None, None]
    assert np.max(np.abs(b - a[mirror][:, :, ::-1]) / w) < 1e-13


def test_hydrostatic_balance(consts):
    """Isothermal fluid under gravity between walls at its temperature
    settles to rest with dp/dy = -rho g r (p = rho T in thermal units, y in
    sites: the pressure gradient theta dp/dy of lattice units balances the
    acceleration g / r), the hydrostatic balance; the stored post-collision velocity is then g/2
    (the step's half-way velocity is zero)."""
    r = consts["r"]
    ly, g0, tau = 32, 2e-4, 0.8
    f = lbm.run_bc(lbm.init(*_uniform(1, ly)), tau, 8000, g=(0.0, -g0), walls=True)
    f2 = lbm.run_bc(f, tau, 50, g=(0.0, -g0), walls=True)
    w = consts["w"][:, None, None]
    assert np.max(np.abs(f2 - f) / w) < 1e-10          # stationary
    rho, ux, uy, T = (a[0] for a in lbm.moments(f))
    p = rho * T
    dp = (p[2:] - p[:-2]) / 2.0
    inner = slice(5, ly - 7)                             # rows 6 .. ly-7
    ratio = dp[inner] / (-rho[1:-1][inner] * g0 * r)
    assert np.all(np.abs(ratio - 1.0) < 2e-3), ratio
    assert np.max(np.abs(uy - (-g0) / 2)) < 0.1 * g0
    assert np.max(np.abs(ux)) < 1e-12


def test_force_driven_channel_flow_curvature(consts):
    """Plane Poiseuille flow: a force g along x between walls at rest gives
    a parabolic velocity profile of curvature -g / nu (thermal units per
    site^2), nu = theta T (tau - 1/2)."""
    theta = consts["theta"]
    ly, g0, tau = 32, 1e-6, 0.8
    f = lbm.run_bc(lbm.init(*_uniform(1, ly)), tau, 8000, g=(g0, 0.0), walls=True)
    rho, ux, uy, T = (a[0] for a in lbm.moments(f))
    y = np.arange(ly)
    inner = slice(4, ly - 4)
    c2 = np.polyfit(y[inner], ux[inner], 2)
    nu = theta * 1.0 * (tau - 0.5)
    assert abs(2 * c2[0] / (-g0 / nu) - 1.0) < 1e-3
    # the profile is symmetric about the channel's centre line
    assert np.max(np.abs(ux - ux[::-1])) < 1e-6 * np.max(ux)


def test_heat_conduction_between_walls():
    """Walls at different temperatures, no force: the fluid comes to rest at
    uniform pressure with a linear temperature profile (the conductivity is
    proportional to p, uniform), falling from the bottom wall's temperature
    to the top's (within the walls' temperature jumps)."""
    ly, tb, tt = 32, 1.02, 0.98
    f = lbm.run_bc(lbm.init(*_uniform(1, ly)), 0.8, 8000, walls=True, t_bottom=tb, t_top=tt)
    rho, ux, uy, T = (a[0] for a in lbm.moments(f))
    y = np.arange(ly)
    inner = slice(6, ly - 6)                             # outside the walls' kinetic layers
    c1 = np.polyfit(y[inner], T[inner], 1)
    drop = (tt - tb)
    assert np.max(np.abs(np.polyval(c1, y[inner]) - T[inner])) < 1e-3 * abs(drop)
    assert 0.9 < c1[0] * ly / drop <= 1.0
    p = rho * T
    assert np.ptp(p[inner]) < 1e-5
    assert np.max(np.abs(uy)) < 1e-4 and np.max(np.abs(ux)) < 1e-12
