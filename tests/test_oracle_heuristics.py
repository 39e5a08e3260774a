"""Pins for the paper's geometric samplers (distance, nearest neighbours): the
first draw of distance sampling follows weights inversely proportional to the
distance (chi-square over seeds), equal distances reduce it to uniform
selection, nearest-neighbour rows equal a brute-force distance computation
(to the column subsample, and to every column when the node has at most 256),
and the fallback behaves as for the learned sampler."""
import numpy as np
from scipy import stats
from scipy.spatial.distance import cdist

from oracle import heuristics as H
from oracle import proposal as P
from oracle.kernels import GAUSSIAN, Kernel
from oracle.skeleton import skeletonize
from oracle.tree import build_tree
from paper_1409_2802_amd import workloads as W


def test_distance_first_draw_follows_inverse_distance():
    f0 = np.array([0.5, 1.0, 2.0, 4.0, 1.5])
    pool = np.arange(5) * 10
    w = (1.0 / f0) / (1.0 / f0).sum()
    counts = np.zeros(5)
    trials = 6000
    for seed in range(trials):
        counts[H.select_rows_distance(f0, pool, 1, seed, node=5)[0] // 10] += 1
    assert stats.chisquare(counts, trials * w).pvalue > 1e-4
    assert H.select_rows_distance(f0, pool, 7, 0, 5).tolist() == pool.tolist()


def test_distance_with_equal_distances_is_uniform():
    pool = np.arange(8) * 3
    counts = np.zeros(8)
    trials = 4000
    for seed in range(trials):
        for r in H.select_rows_distance(np.full(8, 2.0), pool, 3, seed, node=1):
            counts[r // 3] += 1
    assert stats.chisquare(counts, np.full(8, trials * 3 / 8)).pvalue > 1e-4


def _case():
    X = W.gaussian_mixture(3000, 5, k=6, box=6.0, std=0.5, seed=4)
    return X, build_tree(X, 200)


def test_nearest_rows_by_brute_force():
    X, t = _case()
    Xt = X[t.perm]
    checked_exact = 0
    for a in list(t.level_nodes(t.depth))[:4] + [1, 2]:
        b, e = int(t.begin[a]), int(t.end[a])
        cols = np.arange(b, e)
        if len(cols) > 256:
            cols = cols[:240]           # an internal-node-sized column set, all of it in the subsample
        s = 40
        rows, pool, F = H.heuristic_rows(Xt, t, a, cols, s, 3, H.NEAREST)
        g = P.column_geometry(Xt[cols], 3, a)
        dist = cdist(Xt[pool], g.S).min(axis=1) / g.rho
        want = np.sort(pool[np.lexsort((np.arange(len(pool)), dist))[:s]])
        np.testing.assert_array_equal(rows, want)
        if len(cols) <= 256:            # the subsample is every column: nearest to the source set itself
            true = cdist(Xt[pool], Xt[cols]).min(axis=1)
            np.testing.assert_array_equal(rows, np.sort(pool[np.lexsort((np.arange(len(pool)), true))[:s]]))
            checked_exact += 1
        # no unchosen pool point is nearer than a chosen one
        chosen = np.isin(pool, rows)
        assert dist[chosen].max() <= dist[~chosen].min()
    assert checked_exact >= 2


def test_heuristic_skeletonize_and_fallback():
    X, t = _case()
    k = Kernel(GAUSSIAN, h=1.0)
    uni = skeletonize(X, t, k, tol=1e-6, max_rank=24, num_samples=48, seed=2)
    for kind in (H.DISTANCE, H.NEAREST):
        sk, fell = H.skeletonize_heuristic(X, t, k, 1e-6, 24, 48, 2, kind)
        assert not any(fell.values())
        for a, o in sk.nodes.items():
            b, e = int(t.begin[a]), int(t.end[a])
            assert len(o.rows) == 48 and len(np.unique(o.rows)) == 48
            assert np.all((o.rows < b) | (o.rows >= e))       # far targets only
        # A tolerance of zero sends every node with a nonzero held-out residual to uniform rows.
        sk0, fell0 = H.skeletonize_heuristic(X, t, k, 1e-6, 24, 48, 2, kind, fallback_tol=1e-300)
        leaves = list(t.level_nodes(t.depth))
        assert sum(fell0[a] for a in leaves) >= len(leaves) // 2
        for a in leaves:
            if fell0[a]:
                np.testing.assert_array_equal(sk0.nodes[a].rows, uni.nodes[a].rows)
