"""Pins for the adaptive sample count oracle: the held-out error in closed
form, the two limits of the rule (an infinite threshold is plain
skeletonization, a zero threshold is skeletonization at the cap), the
doubling rule itself, and exactly low-rank blocks (which never need more
rows)."""
import numpy as np

from oracle.adaptive import skeletonize_adaptive
from oracle.kernels import GAUSSIAN, POLYNOMIAL, Kernel
from oracle.proposal import heldout_error
from oracle.sampling import sample_far_rows
from oracle.skeleton import skeletonize
from oracle.tree import build_tree
from paper_1409_2802_amd import workloads as W


def test_heldout_error_closed_forms():
    g = np.random.default_rng(0)
    Ks = g.standard_normal((32, 5))
    P = np.hstack([np.eye(5), g.standard_normal((5, 7))])
    perm = g.permutation(12)
    Kh = np.empty((32, 12))
    Kh[:, perm] = Ks @ P                  # columns perm[:5] are the skeleton, the rest combinations of it
    Pp = np.empty((5, 12))
    Pp[:, perm] = P
    assert heldout_error(Kh, perm[:5], Pp) < 1e-14
    # An empty skeleton represents nothing: relative error exactly 1.
    assert heldout_error(Kh, perm[:0], np.zeros((0, 12))) == 1.0
    # Hand example: K = [[1, 2], [3, 4]], skeleton {0}, P = [1, 1] -> residual [[0, 1], [0, 1]].
    K = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert np.isclose(heldout_error(K, np.array([0]), np.array([[1.0, 1.0]])), np.sqrt(2.0 / 30.0), rtol=1e-15)
    assert heldout_error(np.zeros((4, 3)), np.array([0]), np.zeros((1, 3))) == 0.0


def _setup(n=2048, d=6):
    X = W.gaussian_mixture(n, d, k=8, box=5.0, std=0.6, seed=2)
    return X, build_tree(X, 256)


def test_infinite_threshold_is_plain_skeletonization():
    X, t = _setup()
    k = Kernel(GAUSSIAN, h=0.8)
    base = skeletonize(X, t, k, tol=1e-6, max_rank=24, num_samples=48, seed=3)
    ad, hist = skeletonize_adaptive(X, t, k, tol=1e-6, max_rank=24, num_samples=48, seed=3, adaptive_tol=1e300)
    for a, o in base.nodes.items():
        assert len(hist[a]) == 1
        np.testing.assert_array_equal(ad.nodes[a].rows, o.rows)
        np.testing.assert_array_equal(ad.nodes[a].skel, o.skel)
        np.testing.assert_array_equal(ad.nodes[a].P, o.P)


def test_zero_threshold_is_skeletonization_at_the_cap():
    X, t = _setup()
    k = Kernel(GAUSSIAN, h=0.8)
    cap = 160
    ad, hist = skeletonize_adaptive(X, t, k, tol=1e-6, max_rank=24, num_samples=40, seed=5, adaptive_tol=1e-300,
                                    max_samples=cap)
    at_cap = skeletonize(X, t, k, tol=1e-6, max_rank=24, num_samples=cap, seed=5)
    for a, o in at_cap.nodes.items():
        b, e = int(t.begin[a]), int(t.end[a])
        counts = [nr for nr, _ in hist[a]]
        M = t.N - (e - b)
        assert counts == [min(c, M) for c in (40, 80, 160)]     # 40 -> 80 -> 160 = the cap
        np.testing.assert_array_equal(ad.nodes[a].rows, sample_far_rows(b, e, t.N, cap, 5, a))
        np.testing.assert_array_equal(ad.nodes[a].skel, o.skel)
        np.testing.assert_allclose(ad.nodes[a].P, o.P, rtol=0, atol=0)


def test_doubling_rule():
    X, t = _setup()
    k = Kernel(GAUSSIAN, h=0.6)
    tol_a, s0 = 3e-3, 32
    ad, hist = skeletonize_adaptive(X, t, k, tol=1e-7, max_rank=48, num_samples=s0, seed=1, adaptive_tol=tol_a,
                                    max_samples=300)
    grew = 0
    for a, h in hist.items():
        M = t.N - (int(t.end[a]) - int(t.begin[a]))
        expect = s0
        for i, (nr, err) in enumerate(h):
            assert nr == min(expect, M)
            last = i == len(h) - 1
            can_grow = nr < 300 and nr < M
            assert (err > tol_a and can_grow) == (not last)
            expect = min(2 * expect, 300)
        grew += len(h) > 1
        assert len(ad.nodes[a].rows) == h[-1][0]
    assert grew > 0      # the threshold is tight enough that some nodes double


def test_exactly_low_rank_blocks_never_grow():
    # (x.y / h + 1)^1 has rank <= d + 1, so the ID on any >= d + 1 rows is exact and the held-out error is rounding.
    X, t = _setup(d=4)
    k = Kernel(POLYNOMIAL, h=2.0, p=1)
    ad, hist = skeletonize_adaptive(X, t, k, tol=1e-12, max_rank=16, num_samples=16, seed=0, adaptive_tol=1e-8)
    for a, h in hist.items():
        assert len(h) == 1 and h[0][1] < 1e-10
        assert ad.nodes[a].rank <= 5
