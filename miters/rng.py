"""SplitMix64 pseudo-random generator (Steele, Lea and Flood, OOPSLA 2014).

The paper fixes no generator.  SplitMix64 is used because its output sequence
is fully specified by its published definition, so every seed gives the same
circuits on every machine and Python version.  Integers in ``[0, n)`` come from
rejection sampling, so there is no modulo bias.
"""
import math

_M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by rejection sampling."""
        if n <= 0:
            raise ValueError("below() needs n > 0")
        limit = ((1 << 64) // n) * n
        while True:
            r = self.next_u64()
            if r < limit:
                return r % n

    def between(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (both ends included)."""
        return lo + self.below(hi - lo + 1)

    def bit(self) -> int:
        return self.next_u64() >> 63

    def uniform(self) -> float:
        """Uniform float in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def exponential(self, rate: float) -> float:
        """Exponential draw with the given rate (inter-arrival time of a Poisson stream)."""
        return -math.log1p(-self.uniform()) / rate

    def shuffle(self, xs: list) -> None:
        """In-place Fisher-Yates shuffle."""
        for i in range(len(xs) - 1, 0, -1):
            j = self.below(i + 1)
            xs[i], xs[j] = xs[j], xs[i]
