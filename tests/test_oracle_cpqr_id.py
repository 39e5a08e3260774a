"""Pins for the oracle's interpolative decomposition (Section 2.1.3,
Definition of the ID and Theorem thm_compute_id; Appendix 6.1)."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle.cpqr_id import cpqr, interpolative_decomposition, r22_frobenius
from oracle.kernels import POLYNOMIAL, Kernel, kernel_matrix
from oracle.sampling import floyd_sample
from oracle.theory import id_error_factor


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("shape", [(12, 9), (9, 12), (30, 30)])
def test_full_rank_id_is_exact_and_contains_identity(shape):
    A = _rng(0).standard_normal(shape)
    idd = interpolative_decomposition(A, tol=0.0, max_rank=10 ** 6)
    r = min(shape)
    assert idd.rank == r
    np.testing.assert_allclose(A[:, idd.skel] @ idd.P, A, atol=1e-12 * np.abs(A).max())
    # P has the r x r identity on the skeleton columns (Definition of the ID).
    np.testing.assert_array_equal(idd.P[:, idd.skel], np.eye(r))


def test_residual_equals_r22():
    g = _rng(1)
    A = g.standard_normal((40, 8)) @ g.standard_normal((8, 25)) + 1e-6 * g.standard_normal((40, 25))
    idd = interpolative_decomposition(A, tol=1e-4, max_rank=100)
    res = np.linalg.norm(A - A[:, idd.skel] @ idd.P)
    assert res == pytest.approx(r22_frobenius(A, 1e-4, 100), rel=1e-10)


def test_pivots_and_diagonal_match_lapack_dgeqp3():
    """Columns with well separated norms: Businger-Golub pivots are unambiguous."""
    g = _rng(2)
    A = g.standard_normal((20, 12)) * (2.0 ** -np.arange(12))[None, :]
    A = A[:, g.permutation(12)]
    r, piv, RA, _, _ = cpqr(A, tol=0.0, max_rank=12)
    _, R_ref, piv_ref = scipy.linalg.qr(A, pivoting=True, mode="economic")
    np.testing.assert_array_equal(piv, piv_ref)
    np.testing.assert_allclose(np.abs(np.diag(RA[:12, :12])), np.abs(np.diag(R_ref)), rtol=1e-12)
    np.testing.assert_allclose(np.abs(np.triu(RA[:12])), np.abs(R_ref), rtol=1e-10, atol=1e-13)


def test_rank_rule_finds_exact_rank():
    g = _rng(3)
    A = g.standard_normal((50, 6)) @ g.standard_normal((6, 30))
    idd = interpolative_decomposition(A, tol=1e-10, max_rank=30)
    assert idd.rank == 6
    np.testing.assert_allclose(A[:, idd.skel] @ idd.P, A, atol=1e-10 * np.abs(A).max())


def test_rank_cap_and_zero_matrix():
    A = _rng(4).standard_normal((10, 10))
    assert interpolative_decomposition(A, 1e-12, 3).rank == 3
    assert interpolative_decomposition(np.zeros((5, 4)), 1e-6, 4).rank == 0


def test_id_error_between_svd_tail_and_bound():
    """sigma_{r+1} <= ||A - CP||_2 <= sqrt(1 + n r (n - r)) sigma_{r+1} (Theorem thm_compute_id)."""
    g = _rng(5)
    U, _ = np.linalg.qr(g.standard_normal((60, 40)))
    V, _ = np.linalg.qr(g.standard_normal((40, 40)))
    A = U @ np.diag(10.0 ** -np.linspace(0, 8, 40)) @ V.T
    for tol in (1e-2, 1e-4, 1e-6):
        idd = interpolative_decomposition(A, tol=tol, max_rank=40)
        r = idd.rank
        sv = np.linalg.svd(A, compute_uv=False)
        err = np.linalg.norm(A - A[:, idd.skel] @ idd.P, 2)
        assert sv[r] * (1 - 1e-9) <= err <= id_error_factor(40, r) * sv[r]


def test_tie_break_goes_to_smallest_original_column():
    A = np.zeros((4, 4))
    A[0, 3] = A[1, 1] = 2.0
    A[2, 0] = 1.0
    r, piv, _, _, _ = cpqr(A, tol=0.0, max_rank=4)
    assert piv[0] == 1 and piv[1] == 3


@pytest.mark.parametrize("p,rank", [(2, 15), (3, 35)])
def test_polynomial_kernel_exact_rank_and_sampled_reconstruction(p, rank):
    """(x.y/h + 1)^p in d = 4 has rank C(d + p, p) for generic points, so sampled
    rows reproduce all of K (sigma_{r+1} = 0 in Theorem thm_column_sampling_approx2)."""
    assert math.comb(4 + p, p) == rank
    g = _rng(6)
    X = g.standard_normal((80, 4))      # sources
    Y = g.standard_normal((600, 4))     # targets
    k = Kernel(POLYNOMIAL, h=2.0, p=p)
    rows = np.array(floyd_sample(600, 2 * rank, seed=1, stream=0))
    idd = interpolative_decomposition(kernel_matrix(Y[rows], X, k), tol=1e-11, max_rank=80)
    assert idd.rank == rank
    K = kernel_matrix(Y, X, k)
    rel = np.linalg.norm(K - K[:, idd.skel] @ idd.P) / np.linalg.norm(K)
    assert rel < 1e-9


def test_pivot_validity_checker_of_the_parity_tests():
    """The parity tests accept a GPU pivot order that differs from the oracle's only through a near-tie; the
    checker they use accepts the oracle's own order and rejects a swapped pivot or a wrong stopping point."""
    import sys
    from tests._parity import valid_pivot_sequence
    g = np.random.default_rng(0)
    A = g.standard_normal((40, 30)) @ np.diag(10.0 ** -np.linspace(0, 6, 30))
    o = interpolative_decomposition(A, 1e-4, 30)
    assert valid_pivot_sequence(A, o.piv, o.rank, 1e-4, 30)
    bad = o.piv.copy()
    bad[[0, 1]] = bad[[1, 0]]
    assert not valid_pivot_sequence(A, bad, o.rank, 1e-4, 30)
    assert not valid_pivot_sequence(A, o.piv, o.rank - 1, 1e-4, 30)
    # Two equal columns: either order is a valid pivot sequence.
    B = np.hstack([A[:, :1], A[:, :1], A[:, 1:5]])
    ob = interpolative_decomposition(B, 1e-12, 6)
    swapped = ob.piv.copy()
    i, j = list(swapped).index(0), list(swapped).index(1)
    swapped[[i, j]] = swapped[[j, i]]
    assert valid_pivot_sequence(B, swapped, ob.rank, 1e-12, 6)
