"""Pins for the FMM-style evaluation: every (target leaf, source leaf) pair
covered exactly once by a far pair of their ancestors or a direct pair,
admissibility checked by brute-force distances (and the parents of far pairs
not admissible), identity skeletons and an infinite separation giving the
direct sum, and the separated Laplace sum close to the treecode's."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import fmm as F
from oracle import separation as S
from oracle.direct import direct_sum
from oracle.kernels import GAUSSIAN, LAPLACE, Kernel
from oracle.skeleton import NodeSkeleton, Skeletons
from oracle.tree import build_tree
from paper_1409_2802_amd import workloads as W


def _case(N=500, d=3, leaf=30, seed=7):
    X = W.gaussian_mixture(N, d, k=5, box=4.0, std=0.6, seed=seed)
    return X, build_tree(X, leaf)


def _ancestor(t, leaf, level):
    return ((leaf + 1) >> (t.depth - level)) - 1


@pytest.mark.parametrize("xi", [0.5, 1.0, 2.0])
def test_lists_cover_every_leaf_pair_once(xi):
    X, t = _case()
    Xt = X[t.perm]
    far, near = F.fmm_lists(Xt, t, xi)
    leaves = list(t.level_nodes(t.depth))
    n_far = sum(len(v) for v in far.values())
    assert n_far > 0
    for L in leaves:
        for A in leaves:
            hits = sum(_ancestor(t, A, lev) in far[_ancestor(t, L, lev)] for lev in range(1, t.depth + 1))
            hits += A in near[L]
            assert hits == 1, (L, A)


def _ball(Xt, t, a):
    pts = Xt[t.begin[a]:t.end[a]]
    c = pts.sum(axis=0) / len(pts)
    return c, cdist(pts, c[None]).max()


@pytest.mark.parametrize("xi", [0.8, 1.5])
def test_far_pairs_are_admissible_and_maximal(xi):
    X, t = _case(seed=9)
    Xt = X[t.perm]
    far, _ = F.fmm_lists(Xt, t, xi)

    def brute(b, a):
        cb, rb = _ball(Xt, t, b)
        ca, ra = _ball(Xt, t, a)
        pb, pa = Xt[t.begin[b]:t.end[b]], Xt[t.begin[a]:t.end[a]]
        return (cdist(pb, ca[None]).min() >= xi * ra * (1 - 1e-12)
                and cdist(pa, cb[None]).min() >= xi * rb * (1 - 1e-12))

    for b, srcs in far.items():
        for a in srcs:
            assert a != b and brute(b, a)
            pb, pa = (b - 1) // 2, (a - 1) // 2
            if pb > 0:
                assert pb == pa or not F.admissible(Xt, t, pb, pa, xi)


def _identity_skeletons(t):
    sk = Skeletons()
    for a in range(1, t.num_nodes):
        pts = np.arange(t.begin[a], t.end[a], dtype=np.int64)
        sk.nodes[a] = NodeSkeleton(cols=pts, rows=pts[:0], rank=len(pts), piv=np.arange(len(pts)), skel=pts,
                                   P=np.eye(len(pts)), rho=np.zeros(0), gap=np.ones(0))
    return sk


@pytest.mark.parametrize("kind,xi", [(GAUSSIAN, 0.7), (LAPLACE, 1.0), (LAPLACE, 2.5)])
def test_identity_skeletons_give_the_direct_sum(kind, xi):
    X, t = _case(N=400, d=4, leaf=25, seed=11)
    k = Kernel(kind, h=0.8)
    q = W.charges(t.N, seed=4)
    u, uf = F.fmm_evaluate(X, t, _identity_skeletons(t), k, q, xi)
    ref = direct_sum(X, X, q, k)
    np.testing.assert_allclose(u, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    assert np.abs(uf).max() > 0


def test_infinite_separation_is_the_direct_sum():
    X, t = _case(N=300, d=3, leaf=20, seed=13)
    k = Kernel(GAUSSIAN, h=0.9)
    sk = S.skeletonize_separated(X, t, k, tol=1e-6, max_rank=12, num_samples=24, seed=1, xi=1e300)
    q = W.charges(t.N, seed=6)
    u, uf = F.fmm_evaluate(X, t, sk, k, q, 1e300)
    assert np.all(uf == 0.0)
    ref = direct_sum(X, X, q, k)
    np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_separated_laplace_close_to_treecode():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3000, 3))
    t = build_tree(X, 100)
    k = Kernel(LAPLACE)
    q = W.charges(t.N, seed=1)
    ref = direct_sum(X, X, q, k)
    # xi = 1: pairs of nodes are admissible only when separated both ways, a stricter
    # test than the treecode's per-target one.
    sk = S.skeletonize_separated(X, t, k, tol=1e-8, max_rank=32, num_samples=96, seed=3, xi=1.0)
    u_tc, _ = S.treecode_evaluate(X, t, sk, k, q, 1.0)
    u_fmm, uf = F.fmm_evaluate(X, t, sk, k, q, 1.0)
    e_tc = np.linalg.norm(u_tc - ref) / np.linalg.norm(ref)
    e_fmm = np.linalg.norm(u_fmm - ref) / np.linalg.norm(ref)
    assert np.linalg.norm(uf) > 0.05 * np.linalg.norm(u_fmm)
    assert e_fmm < 1e-3 and e_fmm <= e_tc, (e_fmm, e_tc)


def test_target_subsets_give_the_same_values():
    """With a target subset, the treecode and the FMM-style evaluation skip the
    other targets' sums and return the full evaluation's entries (up to the
    rounding of the library's matrix-vector products, whose blocking depends
    on the number of rows)."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((2000, 3))
    t = build_tree(X, 100)
    k = Kernel(LAPLACE)
    q = W.charges(t.N, seed=2)
    sk = S.skeletonize_separated(X, t, k, tol=1e-8, max_rank=24, num_samples=64, seed=1, xi=1.0)
    tg = W.subset(t.N, 97, seed=5)
    for ev in (S.treecode_evaluate, F.fmm_evaluate):
        u, uf = ev(X, t, sk, k, q, 1.0)
        us, ufs = ev(X, t, sk, k, q, 1.0, targets=tg)
        np.testing.assert_allclose(us, u[tg], rtol=1e-13, atol=1e-13 * np.abs(u).max())
        np.testing.assert_allclose(ufs, uf[tg], rtol=1e-13, atol=1e-13 * np.abs(uf).max())
