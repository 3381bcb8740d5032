"""Philox4x32-10 counter-based generator and the normal/uniform draws HMC uses.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x32 with 10 rounds is defined in J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11:
each round multiplies words 0 and 2 of the counter by two fixed 32-bit
constants, mixes the high halves with the other two words and the key, and
the key is advanced by two Weyl constants between rounds.

Draw conventions (shared, as a specification, with the HIP sampler):
  key     = (seed mod 2^32, seed >> 32)
  counter = (index, chain, trajectory, purpose), purpose 0 = momentum, 1 = accept
  uniform in (0, 1]: ((w0 << 21) | (w1 >> 11)) + 1) * 2^-53
  uniform in [0, 1): ((w2 << 21) | (w3 >> 11)) * 2^-53
  normals (Box-Muller): sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2)
Momentum coordinate i of a chain uses counter index i >> 1 and takes the cos
branch for even i, the sin branch for odd i.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ``ctr`` four uint32, ``key`` two uint32 (Python ints)."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox_vec(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(v, np.uint64) & np.uint64(MASK) for v in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK)
    k1 = np.uint64(int(k1) & MASK)
    m0, m1, msk = np.uint64(M0), np.uint64(M1), np.uint64(MASK)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & msk
        hi1, lo1 = p1 >> np.uint64(32), p1 & msk
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _u53(a, b):
    return ((np.asarray(a, np.uint64) << np.uint64(21)) | (np.asarray(b, np.uint64) >> np.uint64(11))).astype(np.float64)


def momentum_normals(seed, chain, traj, d):
    """Standard normals for momentum coordinates 0..d-1 of one chain."""
    npair = (d + 1) // 2
    idx = np.arange(npair, dtype=np.uint64)
    r0, r1, r2, r3 = philox_vec(idx, np.full(npair, chain), np.full(npair, traj),
                                np.zeros(npair), seed & MASK, seed >> 32)
    u1 = (_u53(r0, r1) + 1.0) * 2.0 ** -53
    u2 = _u53(r2, r3) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * npair)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:d]


def accept_uniform(seed, chain, traj):
    """Uniform in (0, 1] for the accept test of one trajectory of one chain."""
    r0, r1, _, _ = philox4x32_10((0, chain, traj, 1), (seed & MASK, seed >> 32))
    return (float(((r0 << 21) | (r1 >> 11))) + 1.0) * 2.0 ** -53
