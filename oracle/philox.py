"""Philox4x64-10 counter-based generator and Box-Muller normals, in NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x64 is defined in Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): four 64-bit counter words, two 64-bit
key words, ten rounds.  Each round multiplies counter words 0 and 2 by the
two round multipliers, keeps the high and low halves of the 128-bit
products, and mixes the high halves with counter words 1 and 3 and the key;
the key is advanced by two Weyl constants between rounds.

Stream convention used by the sampler (both sides implement it):
  key     = (seed, chain)
  counter = (iteration, stream, block, 0)
  stream 0: momentum refresh, stream 1: Metropolis uniform.
A 64-bit output word w maps to u = ((w >> 12) + 1/2) * 2^-52, which is exact
in FP64 and lies in [2^-53, 1 - 2^-53], inside the open interval (0, 1).
Normals come in fours per block by the Box-Muller transform (Box and Muller,
1958): (u0, u1) -> sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1), and likewise
(u2, u3).
"""

from __future__ import annotations

import numpy as np

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK64 = (1 << 64) - 1
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

STREAM_MOMENTUM = 0
STREAM_UNIFORM = 1


def _mulhilo(m: int, x: np.ndarray):
    """High and low 64-bit halves of the 128-bit product m * x (elementwise)."""
    a_lo = np.uint64(m & 0xFFFFFFFF)
    a_hi = np.uint64(m >> 32)
    b_lo = x & _LO32
    b_hi = x >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (hl & _LO32) + lh
    hi = hh + (hl >> _S32) + (cross >> _S32)
    lo = (cross << _S32) | (ll & _LO32)
    return hi, lo


def philox4x64(counter, key, rounds: int = 10) -> np.ndarray:
    """Philox4x64-R on a batch of counters.

    counter: array [n, 4] of uint64; key: (k0, k1) Python ints.
    Returns [n, 4] uint64."""
    x = np.array(counter, dtype=np.uint64).reshape(-1, 4).copy()
    k0, k1 = int(key[0]) & _MASK64, int(key[1]) & _MASK64
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + _W0) & _MASK64
                k1 = (k1 + _W1) & _MASK64
            hi0, lo0 = _mulhilo(_M0, x[:, 0])
            hi1, lo1 = _mulhilo(_M1, x[:, 2])
            x = np.stack([hi1 ^ x[:, 1] ^ np.uint64(k0), lo1,
                          hi0 ^ x[:, 3] ^ np.uint64(k1), lo0], axis=1)
    return x


def to_uniform(w: np.ndarray) -> np.ndarray:
    """Open-interval (0, 1) doubles from 64-bit words: the top 52 bits plus one
    half, scaled by 2^-52 (every step exact in FP64)."""
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def blocks(seed: int, chain: int, iteration: int, stream: int, n_blocks: int) -> np.ndarray:
    ctr = np.zeros((n_blocks, 4), dtype=np.uint64)
    ctr[:, 0] = np.uint64(iteration)
    ctr[:, 1] = np.uint64(stream)
    ctr[:, 2] = np.arange(n_blocks, dtype=np.uint64)
    return philox4x64(ctr, (seed, chain))


def normals(seed: int, chain: int, iteration: int, n: int) -> np.ndarray:
    """The n standard normals of the momentum refresh of (chain, iteration)."""
    nb = (n + 3) // 4
    u = to_uniform(blocks(seed, chain, iteration, STREAM_MOMENTUM, nb))
    r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
    t0 = 2.0 * np.pi * u[:, 1]
    t1 = 2.0 * np.pi * u[:, 3]
    z = np.stack([r0 * np.cos(t0), r0 * np.sin(t0), r1 * np.cos(t1), r1 * np.sin(t1)], axis=1)
    return z.ravel()[:n]


def metropolis_uniform(seed: int, chain: int, iteration: int) -> float:
    """The uniform of the Metropolis test of (chain, iteration)."""
    return float(to_uniform(blocks(seed, chain, iteration, STREAM_UNIFORM, 1))[0, 0])
