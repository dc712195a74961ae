"""D2Q37 velocity set and quadrature weights, derived from first principles.

TEST INFRASTRUCTURE. This package is the oracle: only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it. The GPU
library never reads anything from here.

Section 3 of the paper names the model: 37 populations per site, each moving
up to three lattice points per time step, with the perfect-gas equation of
state p = rho*T. It does not print the velocity set, the weights or the
lattice scale, so this module reconstructs them:

* Velocity set: all integer vectors c with |c|^2 <= 10. That is exactly 37
  vectors (shells |c|^2 = 0, 1, 2, 4, 5, 8, 9, 10 with 1, 4, 4, 4, 8, 4, 4, 8
  members), and no component exceeds 3, matching the "up to three lattice
  points" of Section 3. Order: lexicographic in (cx, cy); the rest vector is
  index 18 and the opposite of i is 36 - i.
* Weights: one weight per shell, plus the lattice scale theta = 1/r^2, chosen
  so that the weighted velocity moments reproduce those of the unit Gaussian
  up to total degree 9 (odd moments vanish by symmetry; the 9 even
  conditions of degree <= 8 fix 8 weights and theta). The system is solved by
  Newton's method in 50-digit arithmetic and rounded to binary64.
* Thermal units: xi_i = r * c_i, so that sum_i w_i xi_i xi_i = identity.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

Q = 37
DIM = 2
MAX_C2 = 10

# Even moment conditions (a, b): sum_i w_i cx^a cy^b = theta^((a+b)/2) (a-1)!! (b-1)!!
_CONDITIONS = ((0, 0), (2, 0), (4, 0), (2, 2), (6, 0), (4, 2), (8, 0), (6, 2), (4, 4))


def velocities() -> np.ndarray:
    """(37, 2) int array of lattice hops, lexicographic in (cx, cy)."""
    vel = [(cx, cy) for cx in range(-3, 4) for cy in range(-3, 4) if cx * cx + cy * cy <= MAX_C2]
    assert len(vel) == Q
    return np.array(vel, dtype=np.int64)


def shells() -> list[int]:
    c = velocities()
    return sorted(set(int(v) for v in (c * c).sum(axis=1)))


def _double_factorial(n: int) -> int:
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


@functools.lru_cache(maxsize=None)
def solve_quadrature(dps: int = 50):
    """Solve the isotropy conditions; returns (shell weights dict, theta) as mpf."""
    mp.mp.dps = dps
    c = velocities()
    sh = shells()
    sums = []
    for a, b in _CONDITIONS:
        row = []
        for s in sh:
            row.append(mp.fsum(mp.mpf(int(cx)) ** a * mp.mpf(int(cy)) ** b
                               for cx, cy in c if cx * cx + cy * cy == s))
        sums.append(row)

    def residual(*x):
        w, th = x[:-1], x[-1]
        return [mp.fsum(sums[k][j] * w[j] for j in range(len(sh)))
                - th ** ((a + b) // 2) * _double_factorial(a - 1) * _double_factorial(b - 1)
                for k, (a, b) in enumerate(_CONDITIONS)]

    # Starting point: a Gaussian-like decay of the weights with |c|^2.
    x0 = [mp.exp(-mp.mpf(s) / 2) / 4 for s in sh] + [mp.mpf("0.7")]
    sol = mp.findroot(residual, x0, tol=mp.mpf(10) ** (-dps + 5), maxsteps=200)
    w = {s: sol[j] for j, s in enumerate(sh)}
    theta = sol[len(sh)]
    res = max(abs(v) for v in residual(*sol))
    return w, theta, res


@functools.lru_cache(maxsize=None)
def constants():
    """Binary64 model constants: dict with c (37,2) int64, w (37,), r, theta, xi (37,2)."""
    w_sh, theta, _ = solve_quadrature()
    c = velocities()
    r = 1 / mp.sqrt(theta)
    w = np.array([float(w_sh[int(cx * cx + cy * cy)]) for cx, cy in c], dtype=np.float64)
    r64 = float(r)
    xi = np.array([[float(r * int(cx)), float(r * int(cy))] for cx, cy in c], dtype=np.float64)
    return {
        "c": c,
        "w": w,
        "r": r64,
        "theta": float(theta),
        "xi": xi,
        "opposite": np.array([Q - 1 - i for i in range(Q)], dtype=np.int64),
    }
