"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), written from its published definition.

The generator is counter based: output number i (i = 1, 2, ...) of a stream with
seed S is mix64(S + i * GAMMA) mod 2^64, so a block of outputs can be drawn with
numpy in one vectorised step and the scalar and vector forms agree exactly.
"""

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def mix64(z: int) -> int:
    """The SplitMix64 output finaliser (Stafford's variant 13)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(_M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(_M2)
        z ^= z >> np.uint64(31)
    return z


class SplitMix64:
    """A SplitMix64 stream.  ``next()`` returns one draw, ``take(k)`` the next k."""

    def __init__(self, seed: int):
        self.seed = seed & MASK64
        self.count = 0

    def next(self) -> int:
        self.count += 1
        return mix64(self.seed + self.count * GAMMA)

    def take(self, k: int) -> np.ndarray:
        """The next ``k`` draws as a uint64 array (same values as k calls of next())."""
        k = int(k)
        if k <= 0:
            return np.zeros(0, dtype=np.uint64)
        idx = np.arange(self.count + 1, self.count + 1 + k, dtype=np.uint64)
        with np.errstate(over="ignore"):
            state = np.uint64(self.seed) + idx * np.uint64(GAMMA)
        self.count += k
        return _mix64_np(state)
