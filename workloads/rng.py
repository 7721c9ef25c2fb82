"""Counter-based SplitMix64 streams (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).

Every random number a workload needs is drawn here and handed to both the
GPU library and the CPU oracle as plain input arrays; neither side draws
random numbers itself.

Output k of a stream seeded with s is mix64(s + (k + 1) * GOLDEN), where
mix64 is the SplitMix64 finaliser.  Streams are vectorised with NumPy
uint64 arithmetic (wrapping multiplication is the intended behaviour).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser on a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """A sequential view of the counter-based stream: draws continue where
    the previous draw stopped."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.counter = 0

    def next_u64(self, count: int) -> np.ndarray:
        k = np.arange(self.counter + 1, self.counter + 1 + count, dtype=np.uint64)
        self.counter += count
        with np.errstate(over="ignore"):
            return mix64(self.seed + k * GOLDEN)

    def uniform01(self, count: int) -> np.ndarray:
        """u = (x >> 11) * 2^-53, in [0, 1)."""
        return (self.next_u64(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def uniform(self, count: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
        u = self.uniform01(count)
        if lo == -1.0 and hi == 1.0:
            return 2.0 * u - 1.0
        return lo + (hi - lo) * u

    def normal(self, count: int) -> np.ndarray:
        """Box-Muller on pairs of uniforms; 1 - u keeps the log argument in (0, 1]."""
        m = (count + 1) // 2
        u1 = 1.0 - self.uniform01(m)
        u2 = self.uniform01(m)
        rad = np.sqrt(-2.0 * np.log(u1))
        out = np.empty(2 * m)
        out[0::2] = rad * np.cos(2.0 * np.pi * u2)
        out[1::2] = rad * np.sin(2.0 * np.pi * u2)
        return out[:count]

    def exponential(self, count: int, rate: float) -> np.ndarray:
        return -np.log(1.0 - self.uniform01(count)) / rate

    def integers(self, count: int, lo: int, hi: int) -> np.ndarray:
        """Integers in [lo, hi] (inclusive) by scaling a uniform; the bias is
        below 2^-40 for the small ranges used here."""
        u = self.uniform01(count)
        return lo + np.minimum(np.floor(u * (hi - lo + 1)).astype(np.int64), hi - lo)
