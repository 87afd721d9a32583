"""Philox4x32-10 counter-based generator -- TEST INFRASTRUCTURE (oracle side).

Written from the definition of Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC 2011): a 4x32-bit counter and a 2x32-bit key;
each of ten rounds multiplies counter words 0 and 2 by 0xD2511F53 and
0xCD9E8D57 (32x32 -> 64 bit), and forms the new counter
(hi(c2 M1) ^ c1 ^ k0, lo(c2 M1), hi(c0 M0) ^ c3 ^ k1, lo(c0 M0));
the key advances by the Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.
The conversions to uniforms and normals follow the library's documented
convention (two 53-bit uniforms per block; Box-Muller for normals).
"""
from __future__ import annotations

import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in counter)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return (c0, c1, c2, c3)


def block(seed: int, stream: int, step: int, index: int):
    """Block `index` of (seed, stream, step): counter (index lo, index hi, step, stream),
    key (seed lo, seed hi)."""
    return philox4x32_10((index & MASK, (index >> 32) & MASK, step & MASK, stream & MASK),
                         (seed & MASK, (seed >> 32) & MASK))


def uniform_pair(a):
    scale = 2.0 ** -53
    u0 = ((a[0] >> 5) * 67108864.0 + (a[1] >> 6) + 0.5) * scale
    u1 = ((a[2] >> 5) * 67108864.0 + (a[3] >> 6) + 0.5) * scale
    return u0, u1


def normal_pair(a):
    u0, u1 = uniform_pair(a)
    r = math.sqrt(-2.0 * math.log(u0))
    return r * math.cos(2.0 * math.pi * u1), r * math.sin(2.0 * math.pi * u1)


def fill(seed: int, stream: int, step: int, n: int, normal: bool) -> np.ndarray:
    out = np.empty(n)
    for i in range((n + 1) // 2):
        a = block(seed, stream, step, i)
        v = normal_pair(a) if normal else uniform_pair(a)
        out[2 * i] = v[0]
        if 2 * i + 1 < n:
            out[2 * i + 1] = v[1]
    return out


def chain_normals(dim: int, n_chains: int, seed: int, stream: int, step: int) -> np.ndarray:
    """Normal i of chain c: member i mod 2 of the pair of block c ceil(dim/2) + i div 2."""
    per = (dim + 1) // 2
    out = np.empty((n_chains, dim))
    for c in range(n_chains):
        for j in range(per):
            z = normal_pair(block(seed, stream, step, c * per + j))
            out[c, 2 * j] = z[0]
            if 2 * j + 1 < dim:
                out[c, 2 * j + 1] = z[1]
    return out
