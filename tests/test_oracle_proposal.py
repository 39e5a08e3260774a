"""Pins for the learned-proposal oracle: MLP gradients by finite differences,
the Adam step in closed form, ridge leverage by an independent linear solve,
weighted selection frequencies, feature invariances and a hand example."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import proposal as P
from oracle.kernels import LAPLACE, Kernel, kernel_matrix
from oracle.sampling import sample_far_rows


def test_parameter_count():
    assert P.NPARAM == 5313


def test_mlp_gradient_matches_central_differences():
    g = np.random.default_rng(0)
    from paper_1409_2802_amd import workloads as W
    theta = W.mlp_init(3) + 0.01 * g.standard_normal(P.NPARAM)
    Z = g.standard_normal((37, P.NF))
    Z[:, 15] = 1.0
    t = g.standard_normal(37)
    loss, grad = P.mlp_loss_grad(theta, Z, t)
    idx = g.choice(P.NPARAM, size=80, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(P.NPARAM)
        e[i] = h
        fd = (P.mlp_loss_grad(theta + e, Z, t)[0] - P.mlp_loss_grad(theta - e, Z, t)[0]) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-5, abs=1e-8)


def test_adam_first_step_closed_form():
    grad = np.array([0.5, -2.0, 1e-3, 0.0])
    theta = np.array([1.0, 1.0, 1.0, 1.0])
    new, m1, m2 = P.adam_step(theta, np.zeros(4), np.zeros(4), grad, step=1, lr=0.01)
    # After one step mhat = g and vhat = g^2, so the update is lr * g / (|g| + eps).
    np.testing.assert_allclose(new, theta - 0.01 * grad / (np.abs(grad) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * grad)
    np.testing.assert_allclose(m2, 0.001 * grad * grad)


def test_ridge_leverage_against_direct_solve_and_invariants():
    g = np.random.default_rng(1)
    B = g.standard_normal((120, 9)) @ np.diag(10.0 ** -np.arange(9)) @ g.standard_normal((9, 30))
    eps = 1e-3
    lev = P.ridge_leverage(B, eps)
    lam = eps * eps * (B * B).sum()
    M = B.T @ B + lam * np.eye(30)
    direct = np.einsum("ij,ji->i", B, np.linalg.solve(M, B.T))
    np.testing.assert_allclose(lev, direct, rtol=1e-8, atol=1e-14)
    sv = np.linalg.svd(B, compute_uv=False)
    assert lev.sum() == pytest.approx((sv ** 2 / (sv ** 2 + lam)).sum(), rel=1e-10)
    assert lev.min() >= 0 and lev.max() < 1


def test_ridge_leverage_problem_case():
    """Rank-two matrix of Section 3: row 1 = v1, others v2: row 1 has leverage ~1."""
    K = np.vstack([np.eye(6)[0]] + [np.eye(6)[1]] * 199)
    lev = P.ridge_leverage(K, 1e-4)
    assert lev[0] == pytest.approx(1.0, abs=1e-5)
    assert lev[1:].sum() == pytest.approx(1.0, abs=1e-5)
    t = P.leverage_targets(lev)
    assert t[0] > t[1] + 4


def test_es_selection_frequencies_follow_weights():
    scores = np.array([0.0, 1.0, 2.0, -1.0, 0.5])
    pool = np.arange(5) * 10
    w = 0.9 * np.exp(scores) / np.exp(scores).sum() + 0.1 / 5
    counts = np.zeros(5)
    trials = 6000
    for seed in range(trials):
        counts[P.select_rows(scores, pool, 1, seed, node=3)[0] // 10] += 1
    assert stats.chisquare(counts, trials * w).pvalue > 1e-4
    assert P.select_rows(scores, pool, 9, 0, 3).tolist() == pool.tolist()


def test_features_invariant_under_rigid_motion_and_scaling():
    g = np.random.default_rng(2)
    Xc = g.standard_normal((150, 5))
    Y = g.standard_normal((40, 5)) * 3
    F = P.features(Y, P.column_geometry(Xc, seed=1, node=7))
    Q, _ = np.linalg.qr(g.standard_normal((5, 5)))
    shift, scale = g.standard_normal(5), 2.5
    G = P.features((Y @ Q.T) * scale + shift, P.column_geometry((Xc @ Q.T) * scale + shift, seed=1, node=7))
    np.testing.assert_allclose(F, G, rtol=1e-9, atol=1e-9)


def test_features_hand_example():
    Xc = np.array([[0.0, 0.0], [2.0, 0.0]])
    geo = P.column_geometry(Xc, seed=0, node=1)
    assert np.allclose(geo.c, [1.0, 0.0]) and geo.rho == 1.0
    F = P.features(np.array([[4.0, 0.0]]), geo)[0]
    assert F[0] == pytest.approx(3.0)
    assert F[1] == pytest.approx(math.log(3.0))
    np.testing.assert_allclose(F[2:6], [2.0, 4.0, 4.0, 4.0])
    assert F[6] == pytest.approx(3.0)
    assert F[7] == pytest.approx(math.log(2.0))
    # anchors: the first point of the subsample farthest from c (both are at distance 1), then the other one
    assert abs(F[8]) == pytest.approx(3.0) and abs(F[9]) == pytest.approx(3.0)
    assert np.allclose(F[10:15], 0.0) and F[15] == 1.0


def test_leverage_sampling_beats_uniform_on_coherent_laplace_block():
    """The gap the learned proposal is for: a near-singular far field (Laplace,
    d = 12, points on a plane) is captured by leverage-weighted rows but not by
    uniform rows (Section 3, problem case)."""
    from paper_1409_2802_amd import workloads as W
    from oracle.cpqr_id import interpolative_decomposition
    X = W.low_intrinsic(3000, 12, di=3, noise=1e-2, seed=0)
    src = np.argsort(np.linalg.norm(X - X[0], axis=1))[:200]
    tgt = np.setdiff1d(np.arange(3000), src)
    k = Kernel(LAPLACE)
    K = kernel_matrix(X[tgt], X[src], k)
    lev = P.ridge_leverage(K, 1e-4)
    scores = np.log(np.maximum(lev, 1e-300))
    rows_l = P.select_rows(scores, np.arange(len(tgt)), 60, seed=0, node=1)
    rows_u = np.sort(np.random.default_rng(0).choice(len(tgt), 60, replace=False))
    errs = {}
    for name, rows in (("lev", rows_l), ("uni", rows_u)):
        idd = interpolative_decomposition(K[rows], 1e-6, 100)
        errs[name] = np.linalg.norm(K - K[:, idd.skel] @ idd.P) / np.linalg.norm(K)
    assert errs["lev"] < 1e-2 * errs["uni"]


def _hand_theta():
    """A sparse parameter vector whose forward pass is worked out by hand below (flat layout: W1 16 x 64
    row-major at 0, b1 at 1024, W2 64 x 64 row-major at 1088, b2 at 5184, w3 at 5248, b3 at 5312)."""
    th = np.zeros(P.NPARAM)
    th[0 * 64 + 0] = 1.0      # W1[0, 0]
    th[1 * 64 + 1] = -2.0     # W1[1, 1]
    th[0 * 64 + 2] = 0.5      # W1[0, 2]
    th[3 * 64 + 0] = 4.0      # W1[3, 0]
    th[1024 + 0] = 0.25       # b1[0]
    th[1024 + 1] = 1.0        # b1[1]
    th[1024 + 2] = -3.0       # b1[2]
    th[1088 + 0 * 64 + 0] = 1.0    # W2[0, 0]
    th[1088 + 1 * 64 + 0] = 10.0   # W2[1, 0]
    th[1088 + 0 * 64 + 1] = -1.0   # W2[0, 1]
    th[1088 + 2 * 64 + 1] = 3.0    # W2[2, 1]
    th[5184 + 0] = 0.5        # b2[0]
    th[5184 + 1] = 1.0        # b2[1]
    th[5248 + 0] = 2.0        # w3[0]
    th[5248 + 1] = 5.0        # w3[1]
    th[5312] = 0.125          # b3
    return th


def test_mlp_forward_hand_values():
    """Forward pass on hand-worked values, so that a swapped layer, a missing ReLU, a transposed weight or a
    dropped bias each changes an output (the finite-difference pin only checks the gradient against the
    forward pass itself).

    Row 1, z = (2, 1, 0, ...): layer 1 pre-activations a = (2 + 0.25, -2 + 1, 1 - 3) = (2.25, -1, -2) -> ReLU
    (2.25, 0, 0); layer 2: a0 = 2.25 + 10 * 0 + 0.5 = 2.75, a1 = -2.25 + 3 * 0 + 1 = -1.25 -> (2.75, 0);
    output 2 * 2.75 + 5 * 0 + 0.125 = 5.625.
    Row 2, z = (-1, -1, 0, 0.5, ...): layer 1 a = (-1 + 2 + 0.25, 2 + 1, -0.5 - 3) = (1.25, 3, -3.5) -> (1.25,
    3, 0); layer 2: a0 = 1.25 + 30 + 0.5 = 31.75, a1 = -1.25 + 0 + 1 = -0.25 -> (31.75, 0); output 63.625.
    Row 3, z = (0, ..., 0): hidden units b1 -> (0.25, 1, 0); layer 2: a0 = 0.25 + 10 + 0.5 = 10.75, a1 =
    -0.25 + 1 = 0.75; output 21.5 + 3.75 + 0.125 = 25.375."""
    th = _hand_theta()
    Z = np.zeros((3, P.NF))
    Z[0, :2] = [2.0, 1.0]
    Z[1, :4] = [-1.0, -1.0, 0.0, 0.5]
    y, (_, A1, H1, A2, H2) = P.mlp_forward(th, Z)
    np.testing.assert_array_equal(y, [5.625, 63.625, 25.375])
    np.testing.assert_array_equal(A1[0, :3], [2.25, -1.0, -2.0])
    np.testing.assert_array_equal(H1[0, :3], [2.25, 0.0, 0.0])
    np.testing.assert_array_equal(A2[1, :2], [31.75, -0.25])
    np.testing.assert_array_equal(H2[2, :2], [10.75, 0.75])
    assert np.all(A1[:, 3:] == 0) and np.all(A2[:, 2:] == 0)


def test_column_geometry_anchor_order_hand_example():
    """Farthest-point anchors on four points with centroid 0 (n <= 256, so the subsample is every point in
    order). Distances to c: P0 4, P1 sqrt(13.25), P2 3, P3 sqrt(21.25). Anchor 1 = P3 (farthest from c);
    anchor 2 = P0 (farthest from P3: 8.56 against 8.25 and 1.80); anchor 3 = P2 (its distance to the nearer
    anchor is 1.80, P1's is sqrt(1.25)); anchor 4 = P1. Choosing by distance to c each time would give P3, P0,
    P1, P2 instead."""
    Xc = np.array([[4.0, 0.0], [3.5, 1.0], [-3.0, 0.0], [-4.5, -1.0]])
    g = P.column_geometry(Xc, seed=0, node=1)
    np.testing.assert_array_equal(g.c, [0.0, 0.0])
    assert g.rho == pytest.approx(math.sqrt(21.25), rel=1e-15)
    expect = np.zeros((7, 2))
    expect[0] = np.array([-4.5, -1.0]) / math.sqrt(21.25)
    expect[1] = [1.0, 0.0]
    expect[2] = [-1.0, 0.0]
    expect[3] = np.array([3.5, 1.0]) / math.sqrt(13.25)
    np.testing.assert_allclose(g.U, expect, rtol=0, atol=1e-15)
    # Projections of y = (1, 2): f8..f14 = (y - c) . u_k / rho.
    F = P.features(np.array([[1.0, 2.0]]), g)
    rho = math.sqrt(21.25)
    np.testing.assert_allclose(F[0, 8:15], [-6.5 / math.sqrt(21.25) / rho, 1.0 / rho, -1.0 / rho,
                                           5.5 / math.sqrt(13.25) / rho, 0.0, 0.0, 0.0], rtol=1e-14, atol=1e-15)
