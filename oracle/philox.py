"""Counter-based Gaussian probes: Philox4x32-10 and Box-Muller (reference, pure Python/numpy).

TEST INFRASTRUCTURE ONLY (see ``oracle/lsop_oracle.py``).

Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key; each of the
10 rounds multiplies words 0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57
(keeping the high and low halves) and mixes them with words 1, 3 and the key;
the key is advanced by the Weyl increments 0x9E3779B9 and 0xBB67AE85 between
rounds.

The probe block of Alg. 2 is drawn as: probe k, pair t (cells 2t, 2t+1) uses
counter (t mod 2^32, t div 2^32, k, 0) and key (seed mod 2^32, seed div 2^32);
with the first two output words x0, x1: u1 = (x0 + 1/2) 2^-32,
u2 = (x1 + 1/2) 2^-32, and the pair is
sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)  (Box & Muller, 1958).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block of Philox4x32-10 on numpy uint64 arrays holding 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(c, np.uint64) & MASK for c in ctr)
    k0, k1 = (np.asarray(k, np.uint64) & MASK for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = c0 * np.uint64(M0)
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def gaussian_probes(nprobe, n, seed):
    """[nprobe, n] standard normals following the counter layout in the module docstring."""
    out = np.empty((nprobe, n))
    t = np.arange((n + 1) // 2, dtype=np.uint64)
    for k in range(nprobe):
        x0, x1, _, _ = philox4x32_10((t & MASK, t >> np.uint64(32), np.full_like(t, k), np.zeros_like(t)),
                                     (seed & MASK, seed >> 32))
        u1 = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
        u2 = (x1.astype(np.float64) + 0.5) * 2.0 ** -32
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * len(t))
        z[0::2] = r * np.cos(2 * np.pi * u2)
        z[1::2] = r * np.sin(2 * np.pi * u2)
        out[k] = z[:n]
    return out
