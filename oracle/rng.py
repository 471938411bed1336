"""SplitMix64 counter-based generator (Steele, Lea and Flood, OOPSLA 2014).

The only random draw inside the method is the Lanczos start vector of the
eigenvalue estimate (Section 2.3.3).  The HIP library implements the same
published generator on its own; nothing is shared.

Definition: the i-th output (i = 0, 1, ...) of the stream with key k is
    z = k + (i + 1) * 0x9E3779B97F4A7C15            (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9        (mod 2^64)
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB        (mod 2^64)
    out = z ^ (z >> 31)
A uniform double in [0, 1) is (out >> 11) * 2^-53.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(key, count):
    """Outputs 0 .. count-1 of the SplitMix64 stream with the given 64-bit key."""
    with np.errstate(over="ignore"):
        i = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(key & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(key, count):
    """count doubles in [0, 1) from the SplitMix64 stream with the given key."""
    return (splitmix64(key, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def lanczos_start(seed, level, count):
    """Start vector of the Lanczos estimate on one level: entries 2U - 1, key seed + level."""
    return 2.0 * uniform01(seed + level, count) - 1.0
