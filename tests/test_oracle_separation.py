"""Pins for the separated far fields and the treecode traversal: the far set
against a brute-force distance computation, xi = 0 reducing to the plain
method, the traversal covering every source exactly once per target and
applying each skeleton at the highest separated node, exact skeletons giving
the direct sum at any xi, an infinite xi giving the direct sum, and the
separated Laplace far field beating the unseparated one."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import separation as S
from oracle.direct import direct_sum
from oracle.evaluate import evaluate
from oracle.kernels import GAUSSIAN, LAPLACE, Kernel
from oracle.skeleton import NodeSkeleton, Skeletons, skeletonize
from oracle.tree import build_tree
from paper_1409_2802_amd import workloads as W


def _case(N=600, d=3, leaf=40, seed=3):
    X = W.gaussian_mixture(N, d, k=5, box=4.0, std=0.6, seed=seed)
    return X, build_tree(X, leaf)


@pytest.mark.parametrize("xi", [0.0, 0.7, 1.0, 2.0])
def test_far_set_by_brute_force(xi):
    X, t = _case()
    Xt = X[t.perm]
    for a in (1, 2, 5, 12, t.num_nodes - 1):
        b, e = int(t.begin[a]), int(t.end[a])
        pts = Xt[b:e]
        c = pts.sum(axis=0) / len(pts)
        rho = cdist(pts, c[None]).max()
        dist = cdist(Xt, c[None])[:, 0]
        want = [p for p in range(t.N) if (p < b or p >= e) and dist[p] >= xi * rho]
        got = S.separated_far_set(Xt, t, a, xi)
        near_edge = np.abs(dist - xi * rho) <= 1e-9 * max(1.0, xi * rho)
        keep = ~near_edge[got]
        assert np.all(np.diff(got) > 0)
        assert set(got[keep]) == set(p for p in want if not near_edge[p])
        if xi == 0.0:
            np.testing.assert_array_equal(got, np.r_[0:b, e:t.N])


def test_xi_zero_is_the_plain_method():
    X, t = _case()
    k = Kernel(GAUSSIAN, h=1.0)
    plain = skeletonize(X, t, k, tol=1e-7, max_rank=20, num_samples=40, seed=5)
    sep = S.skeletonize_separated(X, t, k, tol=1e-7, max_rank=20, num_samples=40, seed=5, xi=0.0)
    for a, o in plain.nodes.items():
        np.testing.assert_array_equal(sep.nodes[a].rows, o.rows)
        np.testing.assert_array_equal(sep.nodes[a].skel, o.skel)
        np.testing.assert_array_equal(sep.nodes[a].P, o.P)
    q = W.charges(t.N, seed=2)
    u0, f0 = evaluate(X, t, plain, k, q)
    u1, f1 = S.treecode_evaluate(X, t, plain, k, q, xi=0.0)
    np.testing.assert_allclose(u1, u0, rtol=1e-13, atol=1e-13 * np.abs(u0).max())
    np.testing.assert_allclose(f1, f0, rtol=1e-13, atol=1e-13 * np.abs(f0).max())


@pytest.mark.parametrize("xi", [0.0, 0.5, 1.0, 1.5, 3.0])
def test_traversal_partitions_sources(xi):
    X, t = _case(N=500, leaf=30, seed=7)
    Xt = X[t.perm]
    far, near = S.interaction_lists(Xt, t, xi)
    cover = np.zeros((t.N, t.N), dtype=np.int32)     # cover[target, source]
    for a, T in far.items():
        b, e = int(t.begin[a]), int(t.end[a])
        for y in T:
            cover[y, b:e] += 1
    for a, T in near.items():
        b, e = int(t.begin[a]), int(t.end[a])
        for y in T:
            cover[y, b:e] += 1
    assert np.all(cover == 1)
    # Every applied node is separated from its target (brute force); its parent
    # (below the root) is not: the traversal applies the highest separated node.
    for a, T in far.items():
        b, e = int(t.begin[a]), int(t.end[a])
        pts = Xt[b:e]
        c = pts.sum(axis=0) / len(pts)
        rho = cdist(pts, c[None]).max()
        for y in T:
            assert not (b <= y < e)
            assert np.linalg.norm(Xt[y] - c) >= xi * rho * (1 - 1e-12)
        p = (a - 1) // 2
        if p > 0:
            pb, pe = int(t.begin[p]), int(t.end[p])
            pp = Xt[pb:pe]
            pc = pp.sum(axis=0) / len(pp)
            prho = cdist(pp, pc[None]).max()
            for y in T:
                assert (pb <= y < pe) or np.linalg.norm(Xt[y] - pc) < xi * prho * (1 + 1e-12)
    # Each target sums its own leaf directly.
    for a, T in near.items():
        b, e = int(t.begin[a]), int(t.end[a])
        assert set(range(b, e)) <= set(T.tolist())


def _identity_skeletons(t):
    """Every node represented by all of its points with P = I: no compression."""
    sk = Skeletons()
    for a in range(1, t.num_nodes):
        pts = np.arange(t.begin[a], t.end[a], dtype=np.int64)
        sk.nodes[a] = NodeSkeleton(cols=pts, rows=pts[:0], rank=len(pts), piv=np.arange(len(pts)), skel=pts,
                                   P=np.eye(len(pts)), rho=np.zeros(0), gap=np.ones(0))
    return sk


@pytest.mark.parametrize("kind,xi", [(GAUSSIAN, 0.0), (GAUSSIAN, 1.2), (LAPLACE, 0.8), (LAPLACE, 2.0)])
def test_exact_skeletons_give_the_direct_sum(kind, xi):
    X, t = _case(N=400, d=4, leaf=25, seed=9)
    k = Kernel(kind, h=0.8)
    q = W.charges(t.N, seed=4)
    u, _ = S.treecode_evaluate(X, t, _identity_skeletons(t), k, q, xi)
    ref = direct_sum(X, X, q, k)
    np.testing.assert_allclose(u, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_infinite_xi_is_the_direct_sum():
    X, t = _case(N=400, d=3, leaf=25, seed=11)
    k = Kernel(GAUSSIAN, h=0.9)
    sk = S.skeletonize_separated(X, t, k, tol=1e-6, max_rank=16, num_samples=32, seed=1, xi=1e300)
    q = W.charges(t.N, seed=6)
    u, uf = S.treecode_evaluate(X, t, sk, k, q, 1e300)
    assert np.all(uf == 0.0)
    ref = direct_sum(X, X, q, k)
    np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # No point is separated, so every node falls back to the plain rows.
    plain = skeletonize(X, t, k, tol=1e-6, max_rank=16, num_samples=32, seed=1)
    for a in plain.nodes:
        np.testing.assert_array_equal(sk.nodes[a].rows, plain.nodes[a].rows)


def test_separation_helps_the_laplace_kernel():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3000, 4))
    t = build_tree(X, 100)
    k = Kernel(LAPLACE)
    q = W.charges(t.N, seed=1)
    ref = direct_sum(X, X, q, k)
    err = {}
    for xi in (0.0, 2.0):
        sk = S.skeletonize_separated(X, t, k, tol=1e-8, max_rank=24, num_samples=96, seed=3, xi=xi)
        u, _ = S.treecode_evaluate(X, t, sk, k, q, xi)
        err[xi] = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert err[2.0] < 0.1 * err[0.0], err
