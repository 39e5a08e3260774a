"""Pins for closed forms (Section 4.2.1 eq. eqn_silverman_bandwidth; Section 3,
Theorem thm_column_sampling_approx2 and its eps = 1/2 corollary) and for the
leverage scores (Section 3, Definition of statistical leverage)."""
import math
import os

import numpy as np
import pytest

from oracle.kernels import POLYNOMIAL, Kernel, kernel_matrix
from oracle.leverage import pivoted_leverage, row_leverage, row_leverage_eps
from oracle.sampling import floyd_sample
from oracle.theory import epsilon_rank, reconstruction_factor, sample_count, silverman_bandwidth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "silverman_bandwidth.txt")


def test_silverman_bandwidth_matches_printed_tables():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for d, N, h in rows:
        assert round(silverman_bandwidth(int(d), int(N)), 4) == pytest.approx(float(h), abs=1e-12)


def test_eps_half_corollary_constants():
    # (1 + eps)(1 - eps)^-2 = 6 and the sample-count coefficient is below 10.
    assert reconstruction_factor(100, 100, 0.5) ** 2 == pytest.approx(1 + 6.0)
    coeff = 1.0 / math.log(1.5 ** 1.5 / math.exp(0.5))
    assert 9.2 < coeff < 10
    assert sample_count(1000, 0.1, 5, 0.1, 0.5) == pytest.approx(1000 * 0.1 * math.log(100) * coeff)


def test_leverage_invariants_and_hat_matrix():
    g = np.random.default_rng(0)
    K = g.standard_normal((60, 12)) @ g.standard_normal((12, 20))
    lev = row_leverage(K, 12)
    assert lev.sum() == pytest.approx(12.0)
    assert lev.min() >= -1e-15 and lev.max() <= 1 + 1e-12
    assert lev.max() >= 12 / 60
    # Full-rank leverage is the diagonal of the hat matrix K K^+.
    hat = K @ np.linalg.pinv(K)
    np.testing.assert_allclose(lev, np.diag(hat), atol=1e-10)


def test_problem_case_rank_two_matrix():
    """Row 1 is v1, the other rows are v2 (Section 3, "A problem case"): the
    first row has leverage 1, and uniform samples of a few rows miss it."""
    m, n = 400, 10
    v1, v2 = np.eye(n)[0], np.eye(n)[1]
    K = np.vstack([v1] + [v2] * (m - 1))
    lev, r = row_leverage_eps(K, 1e-8)
    assert r == 2
    assert lev[0] == pytest.approx(1.0)
    assert lev[1:].sum() == pytest.approx(1.0)
    misses = sum(0 not in floyd_sample(m, 8, seed=s, stream=0) for s in range(500))
    assert misses > 450


def test_uniform_sampling_bound_monte_carlo():
    """Theorem thm_column_sampling_approx2 at eps = 1/2: with s >= 10 m gamma log(2r/delta),
    ||(I - Pi) A||_2 <= sqrt(1 + 6 m / s) sigma_{r+1} in at least 1 - delta of trials.
    The leading right singular vectors are +-1/sqrt(m) patterns, so gamma = r/m
    exactly, and A has more rows than the sample count so the projection is
    not trivially the identity."""
    g = np.random.default_rng(1)
    n, m, r, delta = 200, 4000, 2, 0.2
    v1 = np.ones(m) / math.sqrt(m)
    v2 = np.where(np.arange(m) % 2 == 0, 1.0, -1.0) / math.sqrt(m)
    V, _ = np.linalg.qr(np.column_stack([v1, v2, g.standard_normal((m, n - 2))]))
    U, _ = np.linalg.qr(g.standard_normal((n, n)))
    sig = np.concatenate([[1.0, 0.5], np.full(n - 2, 1e-3)])
    A = U @ np.diag(sig) @ V.T
    gamma = float((V[:, :r] ** 2).sum(1).max())
    assert gamma == pytest.approx(r / m)
    s = int(math.ceil(10 * m * gamma * math.log(2 * r / delta)))
    assert s < n
    bound = math.sqrt(1 + 6 * m / s) * sig[r]
    fails = 0
    for t in range(40):
        cols = floyd_sample(m, s, seed=t, stream=0)
        Q, _ = np.linalg.qr(A[:, cols])
        err = np.linalg.norm(A - Q @ (Q.T @ A), 2)
        assert err >= sig[s] * (1 - 1e-9)          # Eckart-Young: no rank-s projection beats sigma_{s+1}
        fails += err > bound
    assert fails <= delta * 40


def test_epsilon_rank():
    A = np.diag([1.0, 0.1, 1e-3, 1e-5])
    assert epsilon_rank(A, 1e-2) == 2
    assert epsilon_rank(A, 1e-4) == 3
    assert epsilon_rank(np.zeros((3, 3)), 1e-2) == 0


@pytest.mark.parametrize("p,rank", [(2, 15), (3, 35)])
def test_pivoted_leverage_equals_the_svd_leverage_on_exactly_low_rank_blocks(p, rank):
    """A polynomial kernel block in d = 4 has exact rank C(4 + p, p): the pivoted QR stops there, the
    span of its r skeleton columns is the block's range, and the scores equal the singular-vector
    leverage of Section 3 at that rank."""
    g = np.random.default_rng(p)
    Y, X = g.uniform(-1, 1, (300, 4)), g.uniform(-1, 1, (80, 4))
    B = kernel_matrix(Y, X, Kernel(POLYNOMIAL, h=1.0, c=1.0, p=p))
    lev, r, J, _ = pivoted_leverage(B, 1e-9)
    assert r == rank == math.comb(4 + p, p)
    np.testing.assert_allclose(lev, row_leverage(B, rank), atol=1e-9)
    assert lev.sum() == pytest.approx(rank)


def test_pivoted_leverage_invariants_and_problem_case():
    """Scores lie in [0, 1] and sum to the rank; at full column rank they are the hat-matrix diagonal;
    in the paper's rank-two problem case the first row has leverage 1."""
    g = np.random.default_rng(3)
    K = g.standard_normal((70, 9)) * np.linspace(1, 3, 9)
    lev, r, J, _ = pivoted_leverage(K, 1e-12)
    assert r == 9 and sorted(J) == list(range(9))
    assert lev.min() >= -1e-15 and lev.max() <= 1 + 1e-12
    np.testing.assert_allclose(lev, np.diag(K @ np.linalg.pinv(K)), atol=1e-10)
    m, n = 400, 10
    v1, v2 = np.eye(n)[0], np.eye(n)[1]
    P = np.vstack([v1] + [v2] * (m - 1))
    lev, r, J, _ = pivoted_leverage(P, 1e-8)
    assert r == 2 and lev[0] == pytest.approx(1.0) and lev[1:].sum() == pytest.approx(1.0)
    # A truncated factorization: the first pivot is the column of largest norm, and the scores sum to r.
    D = g.standard_normal((50, 6)) @ np.diag([1.0, 0.5, 1e-3, 1e-5, 1e-7, 1e-9]) @ np.linalg.qr(
        g.standard_normal((6, 6)))[0]
    lev, r, J, _ = pivoted_leverage(D, 1e-4)
    assert J[0] == int(np.argmax(np.linalg.norm(D, axis=0)))
    assert 2 <= r <= 4 and lev.sum() == pytest.approx(r)
