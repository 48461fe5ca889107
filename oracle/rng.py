"""Counter-based SplitMix64 generator (oracle side, test infrastructure only).

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; constants as published by Vigna) advances its state
by the golden-ratio increment 0x9E3779B97F4A7C15 and passes the state through
a fixed 64-bit finaliser.  Used as a counter-based generator, the i-th output
for a given seed is the finaliser applied to seed + (i + 1) * increment.
The device library implements the same published definition on its own; the
eigenvalue-estimate start vector is drawn from it on both sides so that the
two agree without sharing code.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    """First n outputs of SplitMix64 seeded with ``seed`` (uint64 array)."""
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed, n):
    """n doubles in [-1, 1): 2 * (top 53 bits / 2^53) - 1."""
    z = splitmix64(seed, n)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
