"""ctypes binding of the C oracle plus numpy helpers (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Arrays follow the canonical layout of the paper's Listing 1: populations
f[p][x][y] with y contiguous; fields [x][y].
"""
from __future__ import annotations

import ctypes
import functools

import numpy as np

from . import build as _build
from .lattice import Q, constants

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


@functools.lru_cache(maxsize=None)
def _lib():
    lib = ctypes.CDLL(_build.build(force=False))
    i, d = ctypes.c_int, ctypes.c_double
    lib.orc_feq_site.argtypes = [_D, _D, d, d, d, d, _D]
    lib.orc_moments_site.argtypes = [_D, _D, _D, _D, _D, _D]
    lib.orc_collide_site.argtypes = [_D, _D, d, _D]
    lib.orc_init.argtypes = [i, i, _D, _D, _D, _D, _D, _D, _D]
    lib.orc_propagate.argtypes = [i, i, _I64, _D, _D]
    lib.orc_collide.argtypes = [i, i, _D, _D, d, _D]
    lib.orc_run.argtypes = [i, i, _I64, _D, _D, d, i, _D, _D]
    lib.orc_moments.argtypes = [i, i, _D, _D, _D, _D, _D, _D]
    lib.orc_audit.argtypes = [i, i, _D, _D, _D]
    lib.orc_collide_site_force.argtypes = [_D, _D, d, d, d, _D]
    lib.orc_collide_force.argtypes = [i, i, _D, _D, d, d, d, _D]
    lib.orc_propagate_walls.argtypes = [i, i, _I64, _D, _D, d, d, _D, _D, _D]
    lib.orc_run_bc.argtypes = [i, i, _I64, _D, _D, d, d, d, i, d, d, i, _D, _D, _D]
    for fn in (lib.orc_collide_site_force, lib.orc_collide_force, lib.orc_propagate_walls, lib.orc_run_bc):
        fn.restype = None
    lib.orc_set_threads.argtypes = [i]
    lib.orc_set_threads.restype = None
    lib.orc_get_threads.argtypes = []
    lib.orc_get_threads.restype = i
    for fn in (lib.orc_feq_site, lib.orc_moments_site, lib.orc_collide_site, lib.orc_init,
               lib.orc_propagate, lib.orc_collide, lib.orc_run, lib.orc_moments, lib.orc_audit):
        fn.restype = None
    return lib


def set_threads(n: int) -> None:
    """Host threads for the column loops of init, propagate and collide
    (results do not depend on it)."""
    _lib().orc_set_threads(int(n))


def get_threads() -> int:
    return _lib().orc_get_threads()


def _p(a: np.ndarray, t=_D):
    return a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _tables():
    k = constants()
    return _f64(k["xi"]), _f64(k["w"]), np.ascontiguousarray(k["c"], dtype=np.int64)


def feq_site(rho: float, ux: float, uy: float, T: float) -> np.ndarray:
    xi, w, _ = _tables()
    out = np.empty(Q)
    _lib().orc_feq_site(_p(xi), _p(w), rho, ux, uy, T, _p(out))
    return out


def moments_site(f: np.ndarray):
    xi, _, _ = _tables()
    f = _f64(f)
    vals = [ctypes.c_double() for _ in range(4)]
    _lib().orc_moments_site(_p(f), _p(xi), *[ctypes.byref(v) for v in vals])
    return tuple(v.value for v in vals)


def collide_site(f: np.ndarray, tau: float) -> np.ndarray:
    xi, w, _ = _tables()
    out = _f64(f).copy()
    _lib().orc_collide_site(_p(xi), _p(w), tau, _p(out))
    return out


def init(rho, ux, uy, T) -> np.ndarray:
    """f = f_eq(rho, u, T), shape (37, lx, ly)."""
    xi, w, _ = _tables()
    rho, ux, uy, T = (_f64(a) for a in (rho, ux, uy, T))
    lx, ly = rho.shape
    f = np.empty((Q, lx, ly))
    _lib().orc_init(lx, ly, _p(xi), _p(w), _p(rho), _p(ux), _p(uy), _p(T), _p(f))
    return f


def propagate(f: np.ndarray) -> np.ndarray:
    _, _, c = _tables()
    f = _f64(f)
    _, lx, ly = f.shape
    out = np.empty_like(f)
    _lib().orc_propagate(lx, ly, _p(c, _I64), _p(f), _p(out))
    return out


def collide(f: np.ndarray, tau: float) -> np.ndarray:
    xi, w, _ = _tables()
    out = _f64(f).copy()
    _, lx, ly = out.shape
    _lib().orc_collide(lx, ly, _p(xi), _p(w), tau, _p(out))
    return out


def run(f: np.ndarray, tau: float, nsteps: int) -> np.ndarray:
    """nsteps x (propagate; collide)."""
    xi, w, c = _tables()
    out = _f64(f).copy()
    _, lx, ly = out.shape
    tmp = np.empty_like(out)
    _lib().orc_run(lx, ly, _p(c, _I64), _p(xi), _p(w), tau, nsteps, _p(out), _p(tmp))
    return out


def collide_site_force(f: np.ndarray, tau: float, g) -> np.ndarray:
    """Forced BGK collision of one site (equilibrium at u + tau g and
    T + tau (1 - tau) |g|^2 / 2)."""
    xi, w, _ = _tables()
    out = _f64(f).copy()
    _lib().orc_collide_site_force(_p(xi), _p(w), tau, float(g[0]), float(g[1]), _p(out))
    return out


def collide_force(f: np.ndarray, tau: float, g) -> np.ndarray:
    xi, w, _ = _tables()
    out = _f64(f).copy()
    _, lx, ly = out.shape
    _lib().orc_collide_force(lx, ly, _p(xi), _p(w), tau, float(g[0]), float(g[1]), _p(out))
    return out


def propagate_walls(f: np.ndarray, t_bottom: float, t_top: float) -> np.ndarray:
    """Pull propagate, periodic in x, diffuse walls at y = -1/2 (t_bottom)
    and y = LY - 1/2 (t_top)."""
    xi, w, c = _tables()
    f = _f64(f)
    _, lx, ly = f.shape
    out = np.empty_like(f)
    rho_w = np.empty(2 * lx)
    _lib().orc_propagate_walls(lx, ly, _p(c, _I64), _p(xi), _p(w), t_bottom, t_top, _p(f), _p(out), _p(rho_w))
    return out


def run_bc(f: np.ndarray, tau: float, nsteps: int, g=(0.0, 0.0), walls: bool = False, t_bottom: float = 1.0,
           t_top: float = 1.0) -> np.ndarray:
    """nsteps x (propagate, with diffuse walls if `walls`; forced collide)."""
    xi, w, c = _tables()
    out = _f64(f).copy()
    _, lx, ly = out.shape
    tmp = np.empty_like(out)
    rho_w = np.empty(2 * lx)
    _lib().orc_run_bc(lx, ly, _p(c, _I64), _p(xi), _p(w), tau, float(g[0]), float(g[1]), int(bool(walls)),
                      t_bottom, t_top, nsteps, _p(out), _p(tmp), _p(rho_w))
    return out


def moments(f: np.ndarray):
    """(rho, ux, uy, T), each (lx, ly)."""
    xi, _, _ = _tables()
    f = _f64(f)
    _, lx, ly = f.shape
    outs = [np.empty((lx, ly)) for _ in range(4)]
    _lib().orc_moments(lx, ly, _p(xi), _p(f), *[_p(o) for o in outs])
    return tuple(outs)


def audit(f: np.ndarray) -> np.ndarray:
    """Lattice totals (mass, px, py, energy = 1/2 sum f xi^2)."""
    xi, _, _ = _tables()
    f = _f64(f)
    _, lx, ly = f.shape
    out = np.empty(4)
    _lib().orc_audit(lx, ly, _p(xi), _p(f), _p(out))
    return out


def run_window(fields, sites, nsteps: int, tau: float) -> np.ndarray:
    """State after nsteps at the given sites of a periodic lattice that starts
    from the equilibrium of `fields` (rho, ux, uy, T, each [lx][ly]).

    A site's value after n steps depends only on the sites within 3n hops
    (each hop moves at most 3 lattice points per step), so each sample is
    computed on its own (6n+1)^2 window: init, then n times (pull propagate
    into the window shrunk by 3 on every side; site-local collide).
    Returns (len(sites), 37).
    """
    rho, ux, uy, T = (np.asarray(a, dtype=np.float64) for a in fields)
    lx, ly = rho.shape
    c = constants()["c"]
    R = 3 * nsteps
    out = np.empty((len(sites), Q))
    for k, (x0, y0) in enumerate(sites):
        xs = (x0 + np.arange(-R, R + 1)) % lx
        ys = (y0 + np.arange(-R, R + 1)) % ly
        ix = np.ix_(xs, ys)
        win = init(rho[ix], ux[ix], uy[ix], T[ix])
        for _ in range(nsteps):
            size = win.shape[1]
            new = np.empty((Q, size - 6, size - 6))
            for p, (cx, cy) in enumerate(c):
                new[p] = win[p, 3 - cx:size - 3 - cx, 3 - cy:size - 3 - cy]
            win = collide(new, tau)
        out[k] = win[:, 0, 0]
    return out
