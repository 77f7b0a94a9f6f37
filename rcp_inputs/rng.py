"""Counter-based uniform numbers from SplitMix64.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the k-th output (k >= 0) of the stream seeded
with `seed` is mix(seed + (k + 1) * 0x9E3779B97F4A7C15) where mix is the
published 64-bit finaliser.  A position draw is addressed by the counter
k = ((i << 24) | attempt) * 4 + axis, and the uniform is the top 53 bits of
the output times 2^-53.  The same definition is implemented independently
in the oracle (C) and in the library's placement code (C++).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, k):
    """k-th output of the SplitMix64 stream started at `seed` (vectorised)."""
    with np.errstate(over="ignore"):
        k = np.asarray(k, dtype=np.uint64)
        z = np.uint64(seed) + (k + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def counter(i, attempt, axis):
    i = np.asarray(i, dtype=np.uint64)
    return ((i << np.uint64(24)) | np.uint64(attempt)) * np.uint64(4) + np.uint64(axis)


def u01(seed, i, attempt, axis):
    """Uniform in [0, 1) with 53 random bits."""
    z = splitmix64(seed, counter(i, attempt, axis))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_positions(n, L, seed):
    """i.i.d. uniform positions in [0, L)^3 (attempt 0), shape (n, 3)."""
    i = np.arange(n, dtype=np.uint64)
    x = np.empty((n, 3), dtype=np.float64)
    for ax in range(3):
        x[:, ax] = u01(seed, i, 0, ax) * L
    x[x >= L] -= L
    return x
