"""Pins for the oracle's kernels and direct sum (Sections 1, 4.2-4.4)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.direct import direct_sum
from oracle.kernels import GAUSSIAN, LAPLACE, POLYNOMIAL, Kernel, kernel_matrix, sqdist


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_sqdist_matches_scalar_loops():
    g = _rng()
    Y, X = g.standard_normal((5, 7)), g.standard_normal((4, 7))
    ref = [[sum((Y[i, k] - X[j, k]) ** 2 for k in range(7)) for j in range(4)] for i in range(5)]
    np.testing.assert_allclose(sqdist(Y, X), np.array(ref), rtol=1e-15, atol=0)


def test_laplace_closed_forms():
    g = _rng(1)
    for d, expo in ((3, 1), (4, 2), (6, 4)):
        Y, X = g.standard_normal((6, d)), g.standard_normal((5, d))
        r = np.array([[math.dist(y, x) for x in X] for y in Y])
        np.testing.assert_allclose(kernel_matrix(Y, X, Kernel(LAPLACE)), r ** (-expo), rtol=1e-13)


def test_laplace_zero_distance_contributes_nothing():
    X = np.array([[0.0, 1.0, 2.0], [1.0, 1.0, 1.0]])
    K = kernel_matrix(X, X, Kernel(LAPLACE))
    assert K[0, 0] == 0.0 and K[1, 1] == 0.0
    assert K[0, 1] == pytest.approx(1.0 / math.sqrt(2.0))


def test_laplace_d2_is_rejected():
    with pytest.raises(ValueError):
        kernel_matrix(np.zeros((1, 2)), np.ones((1, 2)), Kernel(LAPLACE))


def test_gaussian_values_and_wide_limit():
    y = np.array([[0.0, 0.0]])
    x = np.array([[3.0, 4.0]])
    assert kernel_matrix(y, x, Kernel(GAUSSIAN, h=5.0))[0, 0] == pytest.approx(math.exp(-0.5), rel=1e-15)
    g = _rng(2)
    Y, X = g.standard_normal((4, 5)), g.standard_normal((3, 5))
    np.testing.assert_allclose(kernel_matrix(Y, X, Kernel(GAUSSIAN, h=1e9)), 1.0, rtol=1e-15)


def test_polynomial_degree_one_is_affine_and_degree_two_expands():
    g = _rng(3)
    Y, X = g.standard_normal((4, 6)), g.standard_normal((5, 6))
    G = np.array([[float(np.dot(y, x)) for x in X] for y in Y])
    np.testing.assert_allclose(kernel_matrix(Y, X, Kernel(POLYNOMIAL, h=2.0, p=1)), G / 2.0 + 1.0, rtol=1e-14)
    np.testing.assert_allclose(kernel_matrix(Y, X, Kernel(POLYNOMIAL, h=2.0, p=2)),
                               G * G / 4.0 + G + 1.0, rtol=1e-13, atol=1e-14)


def test_direct_sum_exact_rational():
    """Polynomial kernel on small-integer points: the sum is exactly rational."""
    g = _rng(4)
    Y = g.integers(-3, 4, size=(6, 3)).astype(float)
    X = g.integers(-3, 4, size=(8, 3)).astype(float)
    q = g.integers(-5, 6, size=8).astype(float)
    k = Kernel(POLYNOMIAL, h=4.0, c=1.0, p=3)
    exact = []
    for y in Y:
        acc = Fraction(0)
        for x, qj in zip(X, q):
            dot = sum(Fraction(int(a)) * Fraction(int(b)) for a, b in zip(y, x))
            acc += (dot / 4 + 1) ** 3 * Fraction(int(qj))
        exact.append(float(acc))
    np.testing.assert_allclose(direct_sum(Y, X, q, k), exact, rtol=1e-14, atol=1e-12)


def test_direct_sum_gaussian_scalar_loop():
    g = _rng(5)
    Y, X, q = g.random((7, 4)), g.random((9, 4)), g.standard_normal(9)
    ref = [sum(math.exp(-math.dist(y, x) ** 2 / (2 * 0.3 ** 2)) * qj for x, qj in zip(X, q)) for y in Y]
    np.testing.assert_allclose(direct_sum(Y, X, q, Kernel(GAUSSIAN, h=0.3)), ref, rtol=1e-13, atol=1e-15)
