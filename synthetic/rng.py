"""Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), vectorised in numpy.

Value number ``n`` (n = 0, 1, 2, ...) of the stream with seed ``s`` is the SplitMix64
output after ``n + 1`` increments of the state by the golden-ratio constant, i.e.
``mix(s + (n + 1) * 0x9E3779B97F4A7C15)`` with the published finaliser.  Uniform
doubles take the top 53 bits.  Both the oracle tests and the GPU path get their
random inputs from here; the module holds no part of the method's arithmetic.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index) -> np.ndarray:
    """Raw 64-bit outputs for the given counter indices (array-like of ints >= 0)."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, index) -> np.ndarray:
    """Uniform doubles in [0, 1) for the given counter indices."""
    z = splitmix64(seed, index)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_stream(seed: int, n: int, offset: int = 0) -> np.ndarray:
    return uniform(seed, np.arange(offset, offset + n, dtype=np.uint64))
