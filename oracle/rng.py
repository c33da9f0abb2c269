"""Counter-based start vectors (the paper's random_vec in Alg. 10 has no stated
distribution).

READING: element i of a start vector is u(SplitMix64(seed, counter)) mapped to
[-1, 1) with the top 53 bits, where the counter is the U(1) rank (0-based) of
the row's state (of the representative in a momentum sector), and complex
vectors take the real part from counter 2*rank and the imaginary part from
2*rank + 1.  SplitMix64 is the generator published by Steele, Lea and Flood
(OOPSLA 2014, "Fast splittable pseudorandom number generators"): output i of
the stream with seed s is mix64(s + (i + 1) * 0x9E3779B97F4A7C15) with the
finaliser mix64(z) = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31 (all mod 2^64).
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(seed: int, counter: int) -> int:
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & _M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M64
    z ^= z >> 31
    return z


def splitmix64_np(seed: int, counters: np.ndarray) -> np.ndarray:
    """Vectorised splitmix64 over an array of uint64 counters."""
    with np.errstate(over="ignore"):
        c = counters.astype(np.uint64)
        z = np.uint64(seed & _M64) + (c + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def uniform_pm1(seed: int, counters: np.ndarray) -> np.ndarray:
    z = splitmix64_np(seed, counters)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def start_vector(seed: int, row_ranks0: np.ndarray, complex_: bool) -> np.ndarray:
    """Start vector for rows whose states have the given 0-based U(1) ranks."""
    r = np.asarray(row_ranks0, dtype=np.uint64)
    if not complex_:
        return uniform_pm1(seed, r)
    re = uniform_pm1(seed, np.uint64(2) * r)
    im = uniform_pm1(seed, np.uint64(2) * r + np.uint64(1))
    return re + 1j * im
