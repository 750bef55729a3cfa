"""Counter-based Gaussian sketch for the checker (test infrastructure only).

Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from its published definition: a 4-word counter
and a 2-word key; each of the 10 rounds multiplies words 0 and 2 by two fixed
32-bit multipliers, takes the high/low halves, permutes and XORs in the key;
the key is bumped by two Weyl constants between rounds.

Gaussian values use the Box-Muller transform (Box & Muller 1958) on two
uniforms in (0, 1) built from the four output words: the top 52 bits of each
64-bit word pair plus one half, times 2^-52, which is exact in double
precision and lies in [2^-53, 1 - 2^-53].

Element e (row-major) of an m x ell sketch for sketch index s draws from
counter (lo32(e >> 1), hi32(e >> 1), s, 0) with key (lo32(seed), hi32(seed));
even e takes the cosine branch, odd e the sine branch.

Only tests, the smoke entry point and the CPU-baseline leg of the benchmark
may import this package.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox-4x32-10.  All arguments are uint32-valued arrays
    (broadcastable); returns four uint64 arrays holding 32-bit words."""
    c = [np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniform52(lo, hi):
    """(hi:lo) 64-bit word -> uniform double in (0, 1): (top 52 bits + 1/2) 2^-52."""
    w = ((np.asarray(hi, dtype=np.uint64) << np.uint64(32))
         | np.asarray(lo, dtype=np.uint64)) >> np.uint64(12)
    return (w.astype(np.float64) + 0.5) * (2.0 ** -52)


def box_muller(u1, u2):
    """Two independent N(0, 1) values from two uniforms in (0, 1)."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def sketch(seed: int, m: int, ell: int, stream: int = 0) -> np.ndarray:
    """The m x ell Gaussian test matrix Omega (Eq. (14)), float64."""
    e = np.arange(m * ell, dtype=np.uint64)
    g = e >> np.uint64(1)
    seed = np.uint64(seed)
    x0, x1, x2, x3 = philox4x32_10(g & MASK32, g >> np.uint64(32),
                                   np.uint64(stream), np.uint64(0),
                                   seed & MASK32, seed >> np.uint64(32))
    z0, z1 = box_muller(uniform52(x0, x1), uniform52(x2, x3))
    out = np.where((e & np.uint64(1)) == 0, z0, z1)
    return out.reshape(m, ell)
