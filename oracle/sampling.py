"""Uniform sampling of target rows without replacement.

The paper samples rows of K uniformly at random without replacement
(Section 4.1.3, "Uniform sampling"; Theorem thm_column_sampling_approx2 is
stated for sampling without replacement). It names no generator, so the
method fixes one that both sides can reproduce bit for bit:

* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014) used as a counter-based generator: the value for
  (seed, stream, counter) is the first output of a SplitMix64 generator whose
  state is seed XOR (stream << 32) XOR counter.
* Floyd's algorithm (Bentley & Floyd, "Programming pearls: a sample of
  brilliance", CACM 1987) draws s distinct values of {0, ..., M-1}: for
  j = M-s, ..., M-1 take t uniform in {0, ..., j}; keep t if new, else keep j.
  A uniform value in {0, ..., j} is floor(u64 * (j + 1) / 2^64).
* The M candidates are the points outside the node [b, e) in tree order;
  candidate t maps to point t if t < b, else t + (e - b). The result is
  returned in ascending order. Rows are not rescaled: a common scale factor
  changes neither the pivots nor P of the ID.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_next(state: int) -> tuple[int, int]:
    """One SplitMix64 step: returns (new_state, output)."""
    state = (state + GOLDEN_GAMMA) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def counter_u64(seed: int, stream: int, counter: int) -> int:
    """Counter-based 64-bit value for (seed, stream, counter)."""
    x = (seed ^ (stream << 32) ^ counter) & MASK64
    return splitmix64_next(x)[1]


def uniform_below(u64: int, bound: int) -> int:
    """floor(u64 * bound / 2^64), a value in {0, ..., bound - 1}."""
    return (u64 * bound) >> 64


def floyd_sample(M: int, s: int, seed: int, stream: int) -> list[int]:
    """s distinct values of {0, ..., M-1}, ascending (all of them if s >= M)."""
    if s >= M:
        return list(range(M))
    chosen: set[int] = set()
    for j in range(M - s, M):
        t = uniform_below(counter_u64(seed, stream, j), j + 1)
        chosen.add(j if t in chosen else t)
    return sorted(chosen)


def sample_far_rows(b: int, e: int, N: int, s: int, seed: int, node: int) -> np.ndarray:
    """Sampled target rows (tree-order point indices) for the node [b, e)."""
    M = N - (e - b)
    picks = floyd_sample(M, s, seed, node)
    return np.array([t if t < b else t + (e - b) for t in picks], dtype=np.int64)
