"""Pins for the oracle's tree, nested skeletons and far-field evaluation
(Section 2: tree groupings and outgoing representations; eq. e:id)."""
import numpy as np
import pytest

from oracle.direct import direct_sum
from oracle.evaluate import evaluate, exact_far_field, relative_error, sibling
from oracle.kernels import GAUSSIAN, LAPLACE, POLYNOMIAL, Kernel
from oracle.skeleton import skeletonize
from oracle.tree import build_partition, build_tree, tree_depth
from paper_1409_2802_amd import workloads as W


@pytest.mark.parametrize("N,leaf,D", [(1, 4, 0), (4, 4, 0), (5, 4, 1), (1024, 128, 3), (1000, 128, 3), (3, 1, 2)])
def test_depth_rule(N, leaf, D):
    assert tree_depth(N, leaf) == D


def test_tree_is_a_median_split_ball_tree():
    X = W.gaussian_mixture(700, 5, k=6, box=4.0, std=0.5, seed=3)
    t = build_tree(X, 64)
    assert sorted(t.perm.tolist()) == list(range(700))
    for a in range(t.num_nodes):
        b, e = t.begin[a], t.end[a]
        if a < (1 << t.depth) - 1:       # internal node: check its split by brute force
            l, r = 2 * a + 1, 2 * a + 2
            assert t.begin[l] == b and t.end[r] == e and t.end[l] == t.begin[r]
            assert t.end[l] - b == (e - b + 1) // 2
            pts = X[t.perm[b:e]]
            c = pts.mean(axis=0)
            d_c = [float(np.sum((p - c) ** 2)) for p in pts]
            p1 = pts[int(np.argmax(d_c))]
            d_1 = [float(np.sum((p - p1) ** 2)) for p in pts]
            p2 = pts[int(np.argmax(d_1))]
            proj = [float(np.dot(p - c, p2 - p1)) for p in pts]
            nl = t.end[l] - b
            assert max(proj[:nl]) <= min(proj[nl:]) + 1e-12
        if e > b:
            pts = X[t.perm[b:e]]
            np.testing.assert_allclose(t.centroid[a], pts.mean(axis=0), rtol=1e-13, atol=1e-13)
            assert t.radius[a] == pytest.approx(np.sqrt(((pts - t.centroid[a]) ** 2).sum(1)).max())


def test_sibling_cover_partitions_the_far_field():
    t = build_tree(W.uniform_cube(300, 3, seed=1), 20)
    for L in t.level_nodes(t.depth):
        covered = []
        a = L
        while a > 0:
            s = sibling(a)
            covered += list(range(t.begin[s], t.end[s]))
            a = (a - 1) // 2
        outside = [i for i in range(t.N) if not (t.begin[L] <= i < t.end[L])]
        assert sorted(covered) == outside


@pytest.mark.parametrize("k", [Kernel(GAUSSIAN, h=1.0), Kernel(LAPLACE), Kernel(POLYNOMIAL, h=8.0, p=3)])
def test_full_rank_tree_equals_direct_sum(k):
    X = W.gaussian_mixture(384, 6, k=4, box=3.0, std=0.5, seed=0)
    q = W.charges(384, seed=1)
    t = build_tree(X, 24)
    sk = skeletonize(X, t, k, tol=0.0, max_rank=10 ** 6, num_samples=10 ** 6, seed=0)
    u, uf = evaluate(X, t, sk, k, q)
    assert relative_error(u, direct_sum(X, X, q, k)) < 1e-13
    assert relative_error(uf, exact_far_field(X, t, k, q)) < 1e-13


def test_partition_config_error_decreases_with_rank():
    X = W.uniform_cube(1024, 4, seed=0)
    q = W.charges(1024, seed=1)
    t = build_partition(X, 128)
    k = Kernel(GAUSSIAN, h=0.5)
    ex = exact_far_field(X, t, k, q)
    errs = []
    for mr in (16, 64, 128):
        sk = skeletonize(X, t, k, tol=1e-12, max_rank=mr, num_samples=256, seed=0)
        _, uf = evaluate(X, t, sk, k, q)
        errs.append(relative_error(uf[128:], ex[128:]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-8
