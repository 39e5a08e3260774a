"""Closed forms from the paper used as pins and helpers.

* Silverman's KDE bandwidth for standard normal data (Section 4.2.1,
  eq. eqn_silverman_bandwidth): h_S = (4 / (2d + 1))^(1/(d+4)) N^(-1/(d+4)).
* Sample count of Theorem thm_column_sampling_approx2 (eq.
  eqn_sample_complexity) and its error factor (eq.
  eqn_reconstruction_error), plus the eps = 1/2 corollary stated after it.
* The ID error bound of Theorem thm_compute_id: sqrt(1 + n r (n - r)).
* epsilon-rank of a matrix (Section 4.1.3): the least r with
  sigma_{r+1} / sigma_1 < eps.
"""
from __future__ import annotations

import math

import numpy as np


def silverman_bandwidth(d: int, N: int) -> float:
    return (4.0 / (2 * d + 1)) ** (1.0 / (d + 4)) * N ** (-1.0 / (d + 4))


def sample_count(m: int, coherence: float, r: int, delta: float, eps: float) -> float:
    """Lower bound on s in Theorem thm_column_sampling_approx2."""
    return m * coherence * math.log(2 * r / delta) / math.log((1 + eps) ** (1 + eps) / math.exp(eps))


def reconstruction_factor(m: int, s: int, eps: float) -> float:
    """sqrt(1 + (m/s)(1+eps)(1-eps)^-2): the multiple of sigma_{r+1} bounding ||(I-Pi)A||_2."""
    return math.sqrt(1.0 + (m / s) * (1 + eps) / (1 - eps) ** 2)


def id_error_factor(n: int, r: int) -> float:
    return math.sqrt(1.0 + n * r * (n - r))


def epsilon_rank(A: np.ndarray, eps: float) -> int:
    sv = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    if sv.size == 0 or sv[0] == 0.0:
        return 0
    for r in range(sv.size):
        if sv[r] / sv[0] < eps:
            return r
    return int(sv.size)
