"""Kernel functions, evaluated plainly in float64.

Gaussian: exp(-||x - y||^2 / (2 h^2))              Section 4.2, eq. eqn_gaussian_kernel
Laplace:  ||x - y||^(2 - d) for d != 2             Section 4.3 (the d = 2 log branch is not used)
Polynomial: (x^T y / h + c)^p, integer p, c = 1     Section 4.4

Singularity convention for the Laplace kernel: a pair at zero distance
contributes 0 (the paper leaves the self term unspecified; a treecode
evaluates it separately, so it is dropped).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAUSSIAN, LAPLACE, POLYNOMIAL = 0, 1, 2


@dataclass(frozen=True)
class Kernel:
    kind: int
    h: float = 1.0
    c: float = 1.0
    p: int = 1


def sqdist(Y: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances by explicit coordinate differences.

    Y is (m, d), X is (n, d); returns (m, n). No Gram-matrix shortcut, so there
    is no cancellation between ||x||^2 + ||y||^2 and 2 x.y.
    """
    Y = np.asarray(Y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    m, n = Y.shape[0], X.shape[0]
    out = np.empty((m, n))
    if m == 0 or n == 0:
        return out
    rows = max(1, 4_000_000 // max(1, n * Y.shape[1]))
    for a in range(0, m, rows):
        diff = Y[a:a + rows, None, :] - X[None, :, :]
        out[a:a + rows] = np.einsum("mnk,mnk->mn", diff, diff)
    return out


def kernel_matrix(Y: np.ndarray, X: np.ndarray, k: Kernel) -> np.ndarray:
    """K_ij = K(y_i, x_j) for the kernel k, float64, shape (m, n)."""
    Y = np.asarray(Y, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    d = Y.shape[1]
    if k.kind == GAUSSIAN:
        return np.exp(-sqdist(Y, X) / (2.0 * k.h * k.h))
    if k.kind == LAPLACE:
        if d == 2:
            raise ValueError("the d = 2 logarithmic Laplace kernel is not supported")
        r2 = sqdist(Y, X)
        out = np.zeros_like(r2)
        nz = r2 > 0
        out[nz] = r2[nz] ** ((2.0 - d) / 2.0)
        return out
    if k.kind == POLYNOMIAL:
        base = (Y @ X.T) / k.h + k.c
        out = np.ones_like(base)
        for _ in range(k.p):          # integer power by repeated multiplication
            out = out * base
        return out
    raise ValueError(f"unknown kernel kind {k.kind}")
