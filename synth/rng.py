"""SplitMix64 counter-based generator (Steele, Lea and Flood, OOPSLA 2014).

Draw k (k = 0, 1, ...) from seed s is mix(s + (k + 1) * GAMMA mod 2**64), with
mix the published finaliser (xor-shift 30 / 27 / 31 and the two odd
multipliers).  A uniform double in [0, 1) is (x >> 11) * 2**-53.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Return draws offset .. offset+count-1 of the SplitMix64 stream of `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits each."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
