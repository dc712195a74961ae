"""Philox4x32-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC11), and the draws of the learned-collide training pairs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

One Philox4x32 round maps the counter (x0, x1, x2, x3) with key (k0, k1) to
    (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is advanced by the Weyl
constants (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (or ints) of uint32 counters; key: 2 uint32. Returns 4
    uint64 arrays holding the 32-bit outputs."""
    x = [np.asarray(c, dtype=np.uint64) & MASK for c in ctr]
    k0, k1 = np.uint64(key[0] & MASK), np.uint64(key[1] & MASK)
    for r in range(10):
        p0 = np.uint64(M0) * x[0]
        p1 = np.uint64(M1) * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return x


def uniform_from_u32(u) -> np.ndarray:
    """Map a 32-bit word to the open interval (0, 1): the top 23 bits as an
    odd multiple of 2^-24 (exactly representable in FP32)."""
    u = np.asarray(u, dtype=np.uint64)
    return ((u >> np.uint64(9)).astype(np.float64) * 2.0 + 1.0) * 2.0 ** -24


# ---- training-pair draws -----------------------------------------------------
# Pair k of seed s uses key (s mod 2^32, s div 2^32) and the eleven counters
# (k mod 2^32, k div 2^32, j, 0), j = 0..10, giving 44 words w[0..43]:
#   w[0] -> rho = 0.9 + 0.2 U
#   w[1], w[2] -> u = 0.1 sqrt(U1) (cos 2 pi U2, sin 2 pi U2)   (uniform in the disk)
#   w[3] -> T = 0.9 + 0.2 U
#   w[4 + 2q], w[5 + 2q] -> Box-Muller normals n[2q], n[2q+1], q = 0..18 (n[0..36] used)
N_BLOCKS = 11


def pair_words(k: np.ndarray, seed: int) -> np.ndarray:
    """(len(k), 44) uint64 words of pairs k."""
    k = np.asarray(k, dtype=np.uint64)
    key = (seed & MASK, (seed >> 32) & MASK)
    out = np.empty((k.shape[0], 4 * N_BLOCKS), dtype=np.uint64)
    lo, hi = k & np.uint64(MASK), k >> np.uint64(32)
    zero = np.zeros_like(k)
    for j in range(N_BLOCKS):
        r = philox4x32_10((lo, hi, zero + np.uint64(j), zero), key)
        for q in range(4):
            out[:, 4 * j + q] = r[q]
    return out


def pair_draws(k: np.ndarray, seed: int):
    """(rho, ux, uy, T, normals[len(k), 37]) in FP64."""
    w = pair_words(k, seed)
    U = uniform_from_u32(w)
    rho = 0.9 + 0.2 * U[:, 0]
    rad = 0.1 * np.sqrt(U[:, 1])
    ang = 2.0 * np.pi * U[:, 2]
    ux, uy = rad * np.cos(ang), rad * np.sin(ang)
    T = 0.9 + 0.2 * U[:, 3]
    u1 = U[:, 4:42:2]
    u2 = U[:, 5:42:2]
    mag = np.sqrt(-2.0 * np.log(u1))
    n = np.empty((k.shape[0], 38))
    n[:, 0::2] = mag * np.cos(2.0 * np.pi * u2)
    n[:, 1::2] = mag * np.sin(2.0 * np.pi * u2)
    return rho, ux, uy, T, n[:, :37]
