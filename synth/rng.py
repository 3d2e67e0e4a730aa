"""Counter-based SplitMix64 streams for the seeded synthetic inputs.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014, in the form of Vigna's public-domain reference
``splitmix64.c``): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and each output is the state passed through the
xor-shift-multiply finaliser (shifts 30, 27, 31; multipliers
0xBF58476D1CE4E5B9 and 0x94D049BB133111EB).

Because the k-th output depends only on ``seed + (k+1)*gamma`` the stream is
evaluated vectorised in numpy, which keeps generated files identical across
numpy versions (no reliance on numpy's own generators).

This module holds no arithmetic of the rendering method: it only produces the
random numbers from which volumes, cameras and weights are built.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_scalar(state: int) -> tuple[int, int]:
    """One step of the reference generator on Python ints: (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & _MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return state, z ^ (z >> 31)


class SplitMix64:
    """A SplitMix64 stream; draws advance an internal counter."""

    def __init__(self, seed: int):
        self.seed = int(seed) & _MASK64
        self.count = 0

    def uint64(self, n: int) -> np.ndarray:
        k = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        self.count += n
        with np.errstate(over="ignore"):
            states = np.uint64(self.seed) + k * GAMMA
        return mix64(states)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) with 53 random bits each."""
        z = self.uint64(n)
        return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, n: int) -> np.ndarray:
        """Standard normals by Box-Muller (cosine branch), two uniforms each."""
        u = self.uniform(2 * n).reshape(n, 2)
        u1 = 1.0 - u[:, 0]  # (0, 1]: log stays finite
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u[:, 1])


def substream(seed: int, tag: str) -> SplitMix64:
    """An independent stream for one kind of draw (blobs, noise, light, ...)."""
    h = 0
    for ch in tag.encode():
        h = (h * 131 + ch) & _MASK64
    return SplitMix64((int(seed) ^ h) & _MASK64)
