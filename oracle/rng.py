"""Counter-based random numbers the method's sampling step draws (Section 3.1).

The sample of Section 3.1 is a set of uniformly random positions of the
current subproblem.  Positions are a pure function of (seed, subproblem
offset, recursion level, sample index) so that the run is deterministic once
the seed is fixed (Appendix A).  Definition:

    mix64(z)  splitmix64 output function (Steele, Lea & Flood 2014):
              z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
              z ^= z >> 27; z *= 0x94D049BB133111EB
              z ^= z >> 31                                  (mod 2^64)
    h0 = mix64(seed + G); h1 = mix64(h0 ^ offset); h2 = mix64(h1 ^ (level + 1))
    r_i = mix64(h2 + (i + 1) G),  G = 0x9E3779B97F4A7C15
    position_i = floor(r_i * n' / 2^64)

TEST INFRASTRUCTURE ONLY -- see the package docstring.
"""
from __future__ import annotations

import numpy as np

G = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def mix64_int(z: int) -> int:
    z &= M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def splitmix64_stream(state: int, count: int) -> list[int]:
    """The classic splitmix64 generator: state += G; output mix64(state)."""
    out = []
    for _ in range(count):
        state = (state + G) & M64
        out.append(mix64_int(state))
    return out


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * np.uint64(0xBF58476D1CE4E5B9)
        z = z ^ (z >> np.uint64(27))
        z = z * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def sample_base(seed: int, offset: int, level: int) -> int:
    h0 = mix64_int((seed + G) & M64)
    h1 = mix64_int(h0 ^ (offset & M64))
    return mix64_int(h1 ^ ((level + 1) & M64))


def sample_words(seed: int, offset: int, level: int, count: int) -> np.ndarray:
    h2 = sample_base(seed, offset, level)
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64_np(np.uint64(h2) + i * np.uint64(G))


def mulhi64(a: np.ndarray, n: int) -> np.ndarray:
    """floor(a * n / 2^64) for uint64 a and 0 <= n < 2^64, exact (Python ints)."""
    return np.array([(int(x) * n) >> 64 for x in a.tolist()], dtype=np.uint64)


def sample_positions(seed: int, offset: int, level: int, n_sub: int, count: int) -> np.ndarray:
    return mulhi64(sample_words(seed, offset, level, count), n_sub).astype(np.int64)
