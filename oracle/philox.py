"""Philox4x32-10 and Box-Muller, written from their published definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Philox4x32-R (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 4 x 32-bit counter is mixed by R rounds; each round
multiplies two words by fixed odd constants, keeps the high and low halves of
the 64-bit products, and xors the high halves with the other two words and a
round key; the 2 x 32-bit key is bumped by the Weyl constants after every
round.

Normals for the sSVGD noise (eq:noise_term) when the caller passes none:
element e of the [n][d] array uses counter (e // 4 as 64 bits, stream as
64 bits) and key = seed; the four outputs give two Box-Muller pairs
u1 = (x0 + 1) 2^-32, u2 = x1 2^-32, r = sqrt(-2 ln u1),
(r cos 2 pi u2, r sin 2 pi u2), for elements 4q .. 4q+3.
"""
from __future__ import annotations

import math

import numpy as np

MASK = 0xFFFFFFFF
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85


def philox4x32(ctr, key, rounds=10):
    x0, x1, x2, x3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(rounds):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return (x0, x1, x2, x3)


def uint_block(q: int, seed: int, stream: int):
    ctr = (q & MASK, (q >> 32) & MASK, stream & MASK, (stream >> 32) & MASK)
    key = (seed & MASK, (seed >> 32) & MASK)
    return philox4x32(ctr, key)


def box_muller(x0: int, x1: int):
    u1 = (x0 + 1.0) * 2.0 ** -32
    u2 = x1 * 2.0 ** -32
    r = math.sqrt(-2.0 * math.log(u1))
    t = 2.0 * math.pi * u2
    return r * math.cos(t), r * math.sin(t)


def normals(count: int, seed: int, stream: int) -> np.ndarray:
    """First ``count`` standard normals of (seed, stream), in FP64."""
    out = np.empty(count)
    for q in range((count + 3) // 4):
        x = uint_block(q, seed, stream)
        z = box_muller(x[0], x[1]) + box_muller(x[2], x[3])
        for k in range(4):
            e = 4 * q + k
            if e < count:
                out[e] = z[k]
    return out
