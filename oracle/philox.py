"""Counter-based momentum and accept draws (test infrastructure only).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit key go through ten
rounds; each round multiplies counter words 0 and 2 by two fixed odd constants, keeps
the high and low 32-bit halves, and mixes in the other counter words and the key; the
key is bumped by two Weyl constants between rounds.

Stream layout shared with the device generator (both are written independently from this
definition):
  momentum of chain c, iteration t, flat coordinate e (row-major p x K):
      counter = (e // 2, t, c, 0), key = (seed lo 32 bits, seed hi 32 bits)
      words (w0, w1) -> u1, (w2, w3) -> u2, each as ((w_hi << 32 | w_lo) >> 11 + 0.5) * 2^-53
      Box-Muller: r = sqrt(-2 log u1), a = 2 pi u2; even e -> r cos a, odd e -> r sin a
  accept uniform of chain c, iteration t:
      counter = (0, t, c, 1); u = ((w0 << 32 | w1) >> 11 + 0.5) * 2^-53
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32-valued arrays; returns four uint64 arrays < 2^32."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0            # < 2^64, no overflow in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def _u53(hi, lo):
    v = ((hi << np.uint64(32)) | lo) >> np.uint64(11)
    return (v.astype(np.float64) + 0.5) * 2.0 ** -53


def momentum_normals(seed: int, chain: int, it: int, n_coord: int) -> np.ndarray:
    """n_coord standard normals for (chain, iteration), flat coordinate order."""
    q = np.arange((n_coord + 1) // 2, dtype=np.uint64)
    w0, w1, w2, w3 = philox4x32_10(q, it, chain, 0, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u1 = _u53(w0, w1)
    u2 = _u53(w2, w3)
    r = np.sqrt(-2.0 * np.log(u1))
    a = 2.0 * np.pi * u2
    out = np.empty(2 * q.size)
    out[0::2] = r * np.cos(a)
    out[1::2] = r * np.sin(a)
    return out[:n_coord]


def accept_uniform(seed: int, chain: int, it: int) -> float:
    w0, w1, _, _ = philox4x32_10(0, it, chain, 1, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return float(_u53(w0, w1))


def draws(seed: int, chain: int, n_iter: int, p: int, K: int, first_iter: int = 0):
    """(xi [n_iter, p, K], u [n_iter]) for iterations first_iter .. first_iter + n_iter - 1."""
    xi = np.stack([momentum_normals(seed, chain, first_iter + t, p * K).reshape(p, K)
                   for t in range(n_iter)])
    u = np.array([accept_uniform(seed, chain, first_iter + t) for t in range(n_iter)])
    return xi, u
