"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers (points and charges). It holds none of
the method's arithmetic, so both the GPU path and the CPU oracle can be fed
from it without sharing any computation.

Data families (paper, Section 4.1.1, "Data sets"):
  * uniform points in the unit cube (a small, dense parity case);
  * "Normal" data, N(0, I_d);
  * mixtures of Gaussian clusters;
  * "Low intrinsic dimension" data: N(0, I_di) embedded in d dimensions by a
    random orthonormal basis, plus small ambient noise;
  * high-dimensional clustered data: N(0, I_d)/sqrt(d) plus cluster offsets.

Every generator is a pure function of its arguments (numpy PCG64 streams).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cube(n: int, d: int, seed: int = 0) -> np.ndarray:
    """n points uniform in [0, 1]^d, float64, shape (n, d)."""
    return _rng(seed).random((n, d))


def normal(n: int, d: int, seed: int = 0) -> np.ndarray:
    """n points from N(0, I_d) (the paper's "Normal" set)."""
    return _rng(seed).standard_normal((n, d))


def gaussian_mixture(n: int, d: int, k: int = 32, box: float = 10.0,
                     std: float = 0.5, seed: int = 0) -> np.ndarray:
    """Mixture of k equal-weight Gaussian clusters.

    Centres are uniform in [0, box]^d; point i belongs to cluster i mod k and is
    centre + std * N(0, I_d).
    """
    g = _rng(seed)
    centres = g.random((k, d)) * box
    comp = np.arange(n) % k
    return centres[comp] + std * g.standard_normal((n, d))


def low_intrinsic(n: int, d: int, di: int = 8, noise: float = 1e-2,
                  seed: int = 0) -> np.ndarray:
    """Points on a random di-dimensional subspace of R^d plus ambient noise.

    x = B z + noise * g with B an orthonormal d x di basis (QR of a Gaussian
    matrix), z ~ N(0, I_di), g ~ N(0, I_d).
    """
    g = _rng(seed)
    basis, _ = np.linalg.qr(g.standard_normal((d, di)))
    z = g.standard_normal((n, di))
    return z @ basis.T + noise * g.standard_normal((n, d))


def highdim_clusters(n: int, d: int, k: int = 64, offset_norm: float = 3.0,
                     seed: int = 0) -> np.ndarray:
    """x = g / sqrt(d) + c_k, g ~ N(0, I_d), c_k = offset_norm * unit direction.

    Each point picks one of the k offsets uniformly at random.
    """
    g = _rng(seed)
    dirs = g.standard_normal((k, d))
    dirs *= offset_norm / np.linalg.norm(dirs, axis=1, keepdims=True)
    comp = g.integers(0, k, size=n)
    return g.standard_normal((n, d)) / np.sqrt(d) + dirs[comp]


def charges(n: int, seed: int = 1) -> np.ndarray:
    """Densities q ~ N(0, 1), float64, shape (n,)."""
    return _rng(seed).standard_normal(n)


def subset(n_total: int, count: int, seed: int = 2) -> np.ndarray:
    """A sorted seeded subset of `count` distinct indices of range(n_total)."""
    g = _rng(seed)
    return np.sort(g.choice(n_total, size=min(count, n_total), replace=False))


def mlp_init(seed: int = 5) -> np.ndarray:
    """Initial parameters of the 16 -> 64 -> 64 -> 1 proposal network, float64.

    He-normal weights, zero biases, flat in the order W1 (16 x 64, row-major),
    b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1): 5313 values.
    """
    g = _rng(seed)
    W1 = g.standard_normal((16, 64)) * np.sqrt(2.0 / 16)
    W2 = g.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    w3 = g.standard_normal(64) * np.sqrt(1.0 / 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]])
