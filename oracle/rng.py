"""SplitMix64 (Steele, Lea, Flood 2014; constants as published by Vigna).

The sweep starts from a random TT guess and a random residual-projection TT.
Both the oracle and the GPU library draw these from the same counter-based
generator, each with its own implementation of the published definition:

    x_k = mix(seed + (k + 1) * 0x9E3779B97F4A7C15)   (mod 2^64)
    mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
            z *= 0x94D049BB133111EB; z ^= z >> 31
    uniform(-1, 1) = 2 * (x_k >> 11) * 2^-53 - 1

Pinned in tests/test_oracle_tt.py against the published first outputs for
seed 0 (a worked value of the reference implementation).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Raw 64-bit outputs x_offset .. x_{offset+count-1}."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [-1, 1) from the top 53 bits."""
    z = splitmix64(seed, count, offset)
    return 2.0 * (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 1.0


def random_tt(modes, rank: int, seed: int):
    """TT with the given modes and ranks min(rank, full-rank bound) at each bond.

    Entries are consecutive draws, core by core, row-major within a core.
    """
    K = len(modes)
    left = np.cumprod([1] + list(modes))
    right = np.cumprod([1] + list(modes[::-1]))[::-1]
    ranks = [1] + [int(min(rank, left[k], right[k])) for k in range(1, K)] + [1]
    cores, off = [], 0
    for k in range(K):
        cnt = ranks[k] * modes[k] * ranks[k + 1]
        cores.append(uniform_pm1(seed, cnt, off).reshape(ranks[k], modes[k], ranks[k + 1]))
        off += cnt
    return cores
