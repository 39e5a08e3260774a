"""Interpolative decomposition through column-pivoted QR.

The ID of an s x n matrix A is A ~ C P where C holds r columns of A (the
skeleton) and P (r x n) contains the r x r identity as a submatrix
(Section 2.1.3, Definition of the interpolative decomposition). It is computed
from a rank-revealing QR A Pi = Q [R11 R12; 0 R22]: P solves R11 P = R12 and
the skeleton is the first r pivots (Appendix 6.1; Theorem thm_compute_id).

Readings where the paper is silent:
* Pivoting is Businger-Golub column pivoting (largest remaining column norm);
  ties go to the smallest original column index. The trailing column norms
  are recomputed from scratch at every step (no downdating).
* The rank is chosen adaptively: with rho_k the norm of the k-th pivot column
  (= |R_kk|), stop at the first k with rho_k < tol * rho_0, else at
  min(s, n, max_rank); a pivot column of norm exactly zero also stops it (so
  tol = 0 gives the numerical full rank and R11 stays nonsingular). A zero
  matrix gives r = 0. This is the QR analogue of
  the paper's epsilon-rank rule sigma_{r+1} / sigma_1 < eps (Section 4.1.3).
* Householder reflectors use alpha = -sign(x_1) ||x|| with sign(0) = +1; the
  sign choice does not change P.
* R11 is square and nonsingular by the stopping rule, so the "minimum-norm"
  solution of R11 P = R12 is the unique one, found by back substitution.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class ID:
    rank: int
    piv: np.ndarray       # column permutation: piv[k] = original column of pivot k
    R: np.ndarray         # r x n, the first r rows of R in pivoted column order
    T: np.ndarray         # r x (n - r), R11^{-1} R12
    P: np.ndarray         # r x n in original column order
    rho: np.ndarray       # pivot norms rho_0, ..., rho_{r-1} (|R_kk|)
    gap: np.ndarray       # relative gap (best - runner-up) / best of squared norms at each pivot

    @property
    def skel(self) -> np.ndarray:
        return self.piv[: self.rank]


def cpqr(A: np.ndarray, tol: float, max_rank: int):
    """Householder QR with column pivoting, stopped by the rank rule.

    Returns (r, piv, R_full, rho, gap) where R_full is the overwritten s x n array
    whose first r rows hold R (pivoted order) and rows r.. hold R22, and gap
    records, for every pivot examined (including the one that stopped the
    loop), the relative gap between the two largest trailing squared norms.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    s, n = A.shape
    piv = np.arange(n)
    rho = []
    gap = []
    kmax = min(s, n, max_rank)
    rho0 = 0.0
    r = 0
    for k in range(kmax):
        norms2 = np.einsum("ij,ij->j", A[k:, k:], A[k:, k:])
        best = norms2.max()
        cand = np.flatnonzero(norms2 == best) + k
        p = int(cand[np.argmin(piv[cand])])
        rho_k = math.sqrt(norms2[p - k])
        others = np.delete(norms2, p - k)
        gap.append((best - others.max()) / best if others.size and best > 0 else 1.0)
        if k == 0:
            rho0 = rho_k
        if rho_k == 0.0 or rho_k < tol * rho0:
            break
        if p != k:
            A[:, [k, p]] = A[:, [p, k]]
            piv[[k, p]] = piv[[p, k]]
        x = A[k:, k].copy()
        alpha = -math.copysign(rho_k, x[0]) if x[0] != 0.0 else -rho_k
        v = x
        v[0] -= alpha
        vv = float(v @ v)
        if vv > 0.0:
            w = v @ A[k:, k + 1:]
            A[k:, k + 1:] -= np.outer(v, (2.0 / vv) * w)
        A[k, k] = alpha
        A[k + 1:, k] = 0.0
        rho.append(rho_k)
        r = k + 1
    return r, piv, A, np.array(rho), np.array(gap)


def back_substitute(R11: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve R11 T = B for upper-triangular R11, row by row from the bottom."""
    r = R11.shape[0]
    T = np.array(B, dtype=np.float64, copy=True)
    for i in range(r - 1, -1, -1):
        if i + 1 < r:
            T[i] -= R11[i, i + 1:] @ T[i + 1:]
        T[i] /= R11[i, i]
    return T


def interpolative_decomposition(A: np.ndarray, tol: float, max_rank: int) -> ID:
    """Rank-r ID of A: A ~ A[:, skel] @ P (Appendix 6.1)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    r, piv, RA, rho, gap = cpqr(A, tol, max_rank)
    R = RA[:r, :].copy()
    T = back_substitute(R[:, :r], R[:, r:]) if r > 0 else np.zeros((0, n))
    P = np.zeros((r, n))
    P[np.arange(r), piv[:r]] = 1.0
    P[:, piv[r:]] = T
    return ID(rank=r, piv=piv, R=R, T=T, P=P, rho=rho, gap=gap)


def r22_frobenius(A: np.ndarray, tol: float, max_rank: int) -> float:
    """||R22||_F of the stopped factorization (equals ||A - A[:, J] P||_F)."""
    r, _, RA, _, _ = cpqr(A, tol, max_rank)
    return float(np.linalg.norm(RA[r:, r:]))
