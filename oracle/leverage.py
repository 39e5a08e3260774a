"""Statistical leverage scores (Section 3, Definition of statistical leverage).

For the paper's column-sampling matrix A = K^T, the leverage of column j of A
(row j of K) with respect to rank r is the squared norm of row j of V_r, i.e.
of row j of U_r in K = U Sigma V^T. The coherence is the largest score, and
r/m <= coherence <= 1 (Section 3, after eq. e:gamma_def).

The rank is the epsilon-rank of the block (the paper does not say which r the
labels use). "Parity unpinned" does not apply: the scores are pinned by their
invariants (sum = r, range [0, 1]) and by the paper's rank-two problem case.
"""
from __future__ import annotations

import numpy as np

from .theory import epsilon_rank


def row_leverage(K: np.ndarray, r: int) -> np.ndarray:
    """Leverage of every row of K with respect to its best rank-r approximation."""
    K = np.asarray(K, dtype=np.float64)
    if r == 0:
        return np.zeros(K.shape[0])
    U, _, _ = np.linalg.svd(K, full_matrices=False)
    return (U[:, :r] ** 2).sum(axis=1)


def row_leverage_eps(K: np.ndarray, eps: float) -> tuple[np.ndarray, int]:
    r = epsilon_rank(K, eps)
    return row_leverage(K, r), r
