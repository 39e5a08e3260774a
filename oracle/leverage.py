"""Statistical leverage scores (Section 3, Definition of statistical leverage).

For the paper's column-sampling matrix A = K^T, the leverage of column j of A
(row j of K) with respect to rank r is the squared norm of row j of V_r, i.e.
of row j of U_r in K = U Sigma V^T. The coherence is the largest score, and
r/m <= coherence <= 1 (Section 3, after eq. e:gamma_def).

The rank is the epsilon-rank of the block (the paper does not say which r the
labels use).

pivoted_leverage is the same quantity from the method's own factorization:
the column-pivoted QR of the block (the rank rule and pivoting of
cpqr_id.cpqr, tol = eps, no rank cap) picks r columns J, and the scores are
the squared row norms of an orthonormal basis Q_r of span(B(:, J)). When the
block has exact rank r the two subspaces coincide and so do the scores. "Parity unpinned" does not apply: the scores are pinned by their
invariants (sum = r, range [0, 1]) and by the paper's rank-two problem case.
"""
from __future__ import annotations

import numpy as np

from .cpqr_id import cpqr
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


def pivoted_leverage(B: np.ndarray, eps: float):
    """(scores, r, J, gap): squared row norms of Q_r, Q_r an orthonormal basis of the first r pivot
    columns of the column-pivoted QR of B stopped at rho_k < eps rho_0; gap as in cpqr."""
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    r, piv, _, _, gap = cpqr(B, eps, n)
    J = piv[:r].copy()
    if r == 0:
        return np.zeros(m), 0, J, gap
    Q, _ = np.linalg.qr(B[:, J])
    return (Q * Q).sum(axis=1), r, J, gap
