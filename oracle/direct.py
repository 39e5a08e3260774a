"""Direct kernel summation (Section 1, eq. e:sum): u_i = sum_j K(y_i, x_j) q_j."""
from __future__ import annotations

import numpy as np

from .kernels import Kernel, kernel_matrix


def direct_sum(Y: np.ndarray, X: np.ndarray, q: np.ndarray, k: Kernel,
               block: int = 256) -> np.ndarray:
    """u = K q with K the m x n kernel matrix, formed block of targets by block."""
    Y = np.asarray(Y, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    u = np.zeros(Y.shape[0])
    for a in range(0, Y.shape[0], block):
        u[a:a + block] = kernel_matrix(Y[a:a + block], X, k) @ q
    return u


def direct_abs_sum(Y: np.ndarray, X: np.ndarray, q: np.ndarray, k: Kernel,
                   block: int = 256) -> np.ndarray:
    """sum_j |K_ij q_j| per target: the scale of each sum, used to bound rounding."""
    Y = np.asarray(Y, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    out = np.zeros(Y.shape[0])
    for a in range(0, Y.shape[0], block):
        out[a:a + block] = np.abs(kernel_matrix(Y[a:a + block], X, k)) @ np.abs(q)
    return out
