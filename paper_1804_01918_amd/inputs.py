"""Seeded synthetic initial states for the D2Q37 lattice.

This module only draws random numbers and lays out the macroscopic fields of
the initial states; it holds none of the method's arithmetic. Both the GPU
path and the oracle start from the FP64 fields it returns.

Generator: NumPy's PCG64 (``numpy.random.default_rng(seed)``), float64
standard normals, arrays in C order [x][y] (x outer, y contiguous, the
site order of the paper's Listing 1). Velocities and temperatures are in
thermal units (u in units of the reference thermal speed, T relative to the
reference temperature).
"""
from __future__ import annotations

import numpy as np

FIELDS = ("rho", "ux", "uy", "T")


def random_equilibrium(lx: int, ly: int, seed: int = 0, amp: float = 0.01):
    """rho = 1 + amp N, u = amp N per component, T = 1 + amp N; drawn in the
    order rho, ux, uy, T."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal((lx, ly))
    ux = amp * rng.standard_normal((lx, ly))
    uy = amp * rng.standard_normal((lx, ly))
    T = 1.0 + amp * rng.standard_normal((lx, ly))
    return rho, ux, uy, T


def shear_wave(lx: int, ly: int, seed: int = 0, u0: float = 0.05, noise: float = 1e-4, T0: float = 1.0):
    """u_x = u0 sin(2 pi y / ly), rho = 1, T = T0, plus noise N(0,1) added to
    u_x then u_y (draw order u_x, u_y)."""
    rng = np.random.default_rng(seed)
    y = np.arange(ly, dtype=np.float64)
    ux = np.broadcast_to(u0 * np.sin(2.0 * np.pi * y / ly), (lx, ly)).copy()
    uy = np.zeros((lx, ly))
    if noise:
        ux += noise * rng.standard_normal((lx, ly))
        uy += noise * rng.standard_normal((lx, ly))
    rho = np.ones((lx, ly))
    T = np.full((lx, ly), T0)
    return rho, ux, uy, T


def rayleigh_taylor(lx: int, ly: int, seed: int = 0, dT: float = 0.05, amp: float = 0.02,
                    noise: float = 1e-4):
    """Thermal interface at y_i(x) = ly/2 + amp*ly*cos(2 pi x / lx): T = 1 + dT
    below it, 1 - dT above, rho = 1/T (uniform pressure rho T = 1), u = noise
    N(0,1) per component (draw order u_x, u_y)."""
    rng = np.random.default_rng(seed)
    x = np.arange(lx, dtype=np.float64)[:, None]
    y = np.arange(ly, dtype=np.float64)[None, :]
    yi = ly / 2.0 + amp * ly * np.cos(2.0 * np.pi * x / lx)
    T = np.where(y < yi, 1.0 + dT, 1.0 - dT) * np.ones((lx, ly))
    rho = 1.0 / T
    ux = noise * rng.standard_normal((lx, ly))
    uy = noise * rng.standard_normal((lx, ly))
    return rho, ux, uy, T


def perturbation(shape, seed: int, amp: float = 1.0) -> np.ndarray:
    """amp * N(0,1) array of the given shape (non-equilibrium test noise)."""
    return amp * np.random.default_rng(seed).standard_normal(shape)


def make_state(kind: str, lx: int, ly: int, seed: int = 0):
    if kind == "random_equilibrium":
        return random_equilibrium(lx, ly, seed)
    if kind == "shear_wave":
        return shear_wave(lx, ly, seed)
    if kind == "rayleigh_taylor":
        return rayleigh_taylor(lx, ly, seed)
    raise ValueError(f"unknown initial state {kind!r}")
