"""End-to-end GPU skeletonization and evaluation against the oracle
(Section 2.2 sampled ID per node; eq. e:id far field; eq. e:sum direct sum)."""
import numpy as np
import pytest
import torch

from oracle.direct import direct_sum as o_direct
from oracle.evaluate import evaluate as o_evaluate
from oracle.evaluate import exact_far_field
from oracle.kernels import GAUSSIAN, LAPLACE, POLYNOMIAL
from oracle.skeleton import skeletonize as o_skeletonize
from oracle.tree import build_partition as o_partition
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from oracle.skeleton import skeletonize_node
from tests._parity import FP64_REL, check_node_fp64, gkernel, gpu_skeletons, okernel, rel, unambiguous

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def compare_nodes(sk, osk, num_nodes, tol):
    """Rows bit-exact; skeleton identical where the oracle's pivots are clear;
    returns how many nodes were compared exactly."""
    exact = 0
    for a in range(1, num_nodes):
        g, o = sk.node(a), osk.nodes[a]
        np.testing.assert_array_equal(g["rows"], o.rows)
        np.testing.assert_array_equal(g["cols"], o.cols)
        if not unambiguous(o, tol):
            return exact, a
        assert g["rank"] == o.rank, f"node {a}"
        np.testing.assert_array_equal(g["skel"], o.skel)
        scale = max(1.0, np.abs(o.P).max())
        np.testing.assert_allclose(g["P"], o.P, atol=1e-8 * scale)
        exact += 1
    return exact, None


def test_partition_config(ffc):
    """One source node of 256 points against the other 1792 (n = 2048, d = 4,
    Gaussian h = 0.5, s = 128, tol 1e-6, rank cap 64)."""
    X = W.uniform_cube(2048, 4, seed=0)
    q = W.charges(2048, seed=1)
    t = ffc.build_partition(X, 256)
    gk, ok = gkernel(GAUSSIAN, h=0.5), okernel(GAUSSIAN, h=0.5)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=64, num_samples=128, seed=0)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    ot = o_partition(X, 256)
    osk = o_skeletonize(X, ot, ok, tol=1e-6, max_rank=64, num_samples=128, seed=0)
    ou, ouf = o_evaluate(X, ot, osk, ok, q)
    exact, stop = compare_nodes(sk, osk, 3, 1e-6)
    assert stop is None
    assert rel(uf.cpu().numpy(), ouf) < FP64_REL
    assert rel(u.cpu().numpy(), ou) < FP64_REL
    # The far-field error of the method itself, for the record (rank cap binds here).
    ex = exact_far_field(X, ot, ok, q)
    assert rel(uf.cpu().numpy()[256:], ex[256:]) < 1e-2


@pytest.mark.parametrize("kind,kw,data,N,d,leaf,tol,mr", [
    (GAUSSIAN, dict(h=1.0), "mixture", 4096, 16, 256, 1e-5, 64),
    (LAPLACE, dict(), "subspace", 3000, 16, 200, 1e-6, 48),
    (POLYNOMIAL, dict(h=2.0, p=2), "uniform", 2500, 5, 160, 1e-9, 40),
    (GAUSSIAN, dict(h=1.5), "highdim", 1200, 300, 150, 1e-4, 32),
])
def test_tree_config(ffc, kind, kw, data, N, d, leaf, tol, mr):
    make = {"mixture": lambda: W.gaussian_mixture(N, d, k=8, box=6.0, std=0.5, seed=0),
            "subspace": lambda: W.low_intrinsic(N, d, di=4, noise=1e-2, seed=0),
            "uniform": lambda: W.uniform_cube(N, d, seed=0),
            "highdim": lambda: W.highdim_clusters(N, d, k=8, seed=0)}[data]
    X = make()
    q = W.charges(N, seed=1)
    gk, ok = gkernel(kind, **kw), okernel(kind, **kw)
    t = ffc.build_tree(X, leaf)
    sk = ffc.skeletonize(t, gk, tol=tol, max_rank=mr, seed=3)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    ot = o_build_tree(X, leaf)
    Xt = X[ot.perm]
    # Every node against the oracle's node from the same columns; a near-tie is accepted as a valid pivoted QR.
    kinds = {"exact": 0, "valid": 0}
    for a in range(1, ot.num_nodes):
        g = sk.node(a)
        o = skeletonize_node(Xt, ot, a, g["cols"].astype(np.int64), ok, tol, mr, 2 * mr, 3)
        kinds[check_node_fp64(g, o, Xt, ok, tol, mr)] += 1
    assert kinds["exact"] >= 1
    # The sums against the oracle's evaluation of the GPU's skeletons, and (where no tie moved a skeleton) of
    # the oracle's own.
    ou, ouf = o_evaluate(X, ot, gpu_skeletons(sk, ot.num_nodes), ok, q)
    assert rel(uf.cpu().numpy(), ouf) < FP64_REL
    assert rel(u.cpu().numpy(), ou) < FP64_REL
    if kinds["valid"] == 0:
        ou2, _ = o_evaluate(X, ot, o_skeletonize(X, ot, ok, tol=tol, max_rank=mr, seed=3), ok, q)
        assert rel(u.cpu().numpy(), ou2) < FP64_REL
    ffc.check_device()


@pytest.mark.parametrize("kind,kw", [(GAUSSIAN, dict(h=1.0)), (LAPLACE, dict()), (POLYNOMIAL, dict(h=3.0, p=3))])
def test_full_rank_equals_direct(ffc, kind, kw):
    """tol = 0 and no rank cap: the compressed sum is the direct sum."""
    X = W.gaussian_mixture(777, 6, k=4, box=3.0, std=0.5, seed=2)
    q = W.charges(777, seed=3)
    gk, ok = gkernel(kind, **kw), okernel(kind, **kw)
    t = ffc.build_tree(X, 50)
    sk = ffc.skeletonize(t, gk, tol=0.0, max_rank=4096, num_samples=4096, seed=0)
    u, _ = ffc.evaluate_sum(t, sk, gk, q)
    ud = ffc.direct_sum(X, X, q, gk)
    ref = o_direct(X, X, q, ok)
    assert rel(u.cpu().numpy(), ref) < 1e-12
    assert rel(ud.cpu().numpy(), ref) < 1e-13


def test_skeleton_reuse_and_determinism(ffc):
    X = W.uniform_cube(3000, 8, seed=5)
    q = W.charges(3000, seed=6)
    gk = gkernel(GAUSSIAN, h=0.7)
    t = ffc.build_tree(X, 128)
    sk = ffc.skeletonize(t, gk, tol=1e-4, max_rank=32, seed=1)
    u1, _ = ffc.evaluate_sum(t, sk, gk, q)
    sk2 = ffc.skeletonize(t, gk, tol=1e-4, max_rank=32, seed=1, reuse=sk)
    assert sk2 is sk
    u2, _ = ffc.evaluate_sum(t, sk, gk, q)
    assert torch.equal(u1, u2)


@pytest.mark.parametrize("N", [1, 50])
def test_single_leaf_tree(ffc, N):
    """Depth 0 (every point in the root leaf): nothing to skeletonize, the far field is empty and the sum is the
    direct sum."""
    X = W.uniform_cube(N, 5, seed=4)
    q = W.charges(N, seed=5)
    gk, ok = gkernel(GAUSSIAN, h=0.8), okernel(GAUSSIAN, h=0.8)
    t = ffc.build_tree(X, 64)
    assert t.depth == 0 and t.num_nodes == 1
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=16)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    assert np.all(uf.cpu().numpy() == 0.0)
    assert rel(u.cpu().numpy(), o_direct(X, X, q, ok)) < 1e-13
    assert sk.stats()["num_nodes"] == 0
