"""SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; constants as published by S. Vigna), used
counter-style: the i-th output (i = 0, 1, ...) of a stream seeded with s is the
mix of s + (i + 1) * golden_gamma modulo 2^64."""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    """First n outputs of SplitMix64 seeded with `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, n):
    """Doubles in [0, 1) from the top 53 bits of each SplitMix64 output."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm(seed, n, amp):
    """n doubles uniform in [-amp, amp)."""
    return amp * (2.0 * uniform01(seed, n) - 1.0)
