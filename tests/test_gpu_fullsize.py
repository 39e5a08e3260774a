"""Parity at the workloads' full sizes, in the configuration bench.py times:
every node of the mixture16 tree (N = 65536, d = 16) and of the separated
Laplace trees (N = 65536, d = 3; treecode at separation 2, FMM-style at 1)
against the oracle's own skeletonization and evaluation (the Laplace sums on
sampled targets); sampled leaves and sampled direct-sum targets of the
d = 1000 and N = 262144 workloads."""
import numpy as np
import pytest
import torch

from oracle.direct import direct_sum as o_direct
from oracle.fmm import fmm_evaluate
from oracle.separation import skeletonize_separated, treecode_evaluate
from oracle.evaluate import evaluate as o_evaluate
from oracle.kernels import GAUSSIAN, LAPLACE, POLYNOMIAL
from oracle.skeleton import skeletonize as o_skeletonize
from oracle.skeleton import skeletonize_node
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from tests._parity import FP64_REL, direct_bound, gkernel, okernel, rel, unambiguous

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def check_node(g, o, tol):
    """Rows bit-exact; skeleton and P where the oracle's pivots are clear. True if compared in full."""
    np.testing.assert_array_equal(g["rows"], o.rows)
    np.testing.assert_array_equal(g["cols"], o.cols)
    if not unambiguous(o, tol):
        return False
    assert g["rank"] == o.rank
    np.testing.assert_array_equal(g["skel"], o.skel)
    np.testing.assert_allclose(g["P"], o.P, atol=1e-8 * max(1.0, np.abs(o.P).max()))
    return True


def test_mixture16_every_node(ffc):
    """The default bench workload: N=65536, d=16, 32 clusters, Gaussian h=1, leaf 512, s=512, rank cap 256,
    tol 1e-5, FP64: all 254 nodes and the far field at every target."""
    X = W.gaussian_mixture(65536, 16, k=32, box=10.0, std=0.5, seed=0)
    q = W.charges(65536, seed=1)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 512)
    sk = ffc.skeletonize(t, gk, tol=1e-5, max_rank=256, num_samples=512, seed=0)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    ot = o_build_tree(X, 512)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    osk = o_skeletonize(X, ot, ok, tol=1e-5, max_rank=256, num_samples=512, seed=0)
    full, stop = 0, None
    for level in range(ot.depth, 0, -1):
        for a in ot.level_nodes(level):
            if stop is not None:
                break
            if check_node(sk.node(a), osk.nodes[a], 1e-5):
                full += 1
            else:
                stop = a   # an ambiguous pivot may change everything above it
    assert full >= (1 << ot.depth), (full, stop)   # at least the whole leaf level
    if stop is None:
        ou, ouf = o_evaluate(X, ot, osk, ok, q)
        assert rel(uf.cpu().numpy(), ouf) < FP64_REL
        assert rel(u.cpu().numpy(), ou) < FP64_REL


@pytest.mark.parametrize("kind,kw", [(POLYNOMIAL, dict(h=1.0, p=3)), (GAUSSIAN, dict(h=1.5))])
def test_highdim1000_sampled(ffc, kind, kw):
    """N=65536, d=1000 (N(0,I)/sqrt(d) + 64 offsets of norm 3), leaf 512, s=512, rank cap 256, tol 1e-4, FP64:
    4 sampled leaves against the oracle, and 48 sampled targets of the direct sum."""
    N, d = 65536, 1000
    X = W.highdim_clusters(N, d, k=64, seed=0)
    q = W.charges(N, seed=1)
    gk, ok = gkernel(kind, **kw), okernel(kind, **kw)
    t = ffc.build_tree(X, 512)
    sk = ffc.skeletonize(t, gk, tol=1e-4, max_rank=256, num_samples=512, seed=0)
    ot = o_build_tree(X, 512)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    Xt = X[ot.perm]
    leaves = list(ot.level_nodes(ot.depth))
    compared = 0
    for a in np.random.default_rng(7).choice(leaves, 4, replace=False):
        cols = np.arange(ot.begin[a], ot.end[a], dtype=np.int64)
        o = skeletonize_node(Xt, ot, int(a), cols, ok, 1e-4, 256, 512, 0)
        compared += check_node(sk.node(int(a)), o, 1e-4)
    assert compared >= 2
    tg = W.subset(N, 48, seed=2)
    Xd = torch.as_tensor(X, device="cuda")
    u = ffc.direct_sum(Xd[tg], Xd, q, gk).cpu().numpy()
    uo = o_direct(X[tg], X, q, ok)
    bound = direct_bound(X[tg], X, q, kind, kw)
    assert np.all(np.abs(u - uo) <= bound)


def test_subspace64_sampled_leaves(ffc):
    """N=262144, d=64 points near an 8-dim subspace, Laplace, leaf 1024, s=512, rank cap 256, tol 1e-6, FP64:
    the tree, and 4 sampled leaves against the oracle."""
    N, d = 262144, 64
    X = W.low_intrinsic(N, d, di=8, noise=1e-2, seed=0)
    gk, ok = gkernel(LAPLACE), okernel(LAPLACE)
    t = ffc.build_tree(X, 1024)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=256, num_samples=512, seed=0)
    ot = o_build_tree(X, 1024)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    Xt = X[ot.perm]
    compared = 0
    for a in np.random.default_rng(8).choice(list(ot.level_nodes(ot.depth)), 4, replace=False):
        cols = np.arange(ot.begin[a], ot.end[a], dtype=np.int64)
        o = skeletonize_node(Xt, ot, int(a), cols, ok, 1e-6, 256, 512, 0)
        compared += check_node(sk.node(int(a)), o, 1e-6)
    assert compared >= 2


@pytest.mark.parametrize("xi,fmm", [(2.0, False), (1.0, True)])
def test_separated_laplace_every_node(ffc, xi, fmm):
    """The separated3 (treecode, xi = 2) and fmm3 (FMM-style, xi = 1) workloads: N=65536, d=3 N(0,I), Laplace
    1/r, leaf 256, s=256, rank cap 128, tol 1e-6, FP64: all 510 nodes, then the far field and the whole sum at
    512 sampled targets."""
    X = W.normal(65536, 3, seed=0)
    q = W.charges(65536, seed=1)
    gk, ok = gkernel(LAPLACE), okernel(LAPLACE)
    t = ffc.build_tree(X, 256)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=128, num_samples=256, seed=0, separation=xi)
    u, uf = (ffc.evaluate_fmm if fmm else ffc.evaluate_sum)(t, sk, gk, q)
    u, uf = u.cpu().numpy(), uf.cpu().numpy()
    ot = o_build_tree(X, 256)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    osk = skeletonize_separated(X, ot, ok, 1e-6, 128, 256, 0, xi)
    full, stop = 0, None
    for level in range(ot.depth, 0, -1):
        for a in ot.level_nodes(level):
            if stop is not None:
                break
            if check_node(sk.node(a), osk.nodes[a], 1e-6):
                full += 1
            else:
                stop = a
    assert full >= (1 << ot.depth), (full, stop)
    print(f"xi={xi} fmm={fmm}: {full} nodes compared in full, first ambiguous node {stop}")
    if stop is None:
        tg = W.subset(65536, 512, seed=2)
        ou, ouf = (fmm_evaluate if fmm else treecode_evaluate)(X, ot, osk, ok, q, xi, targets=tg)
        assert rel(uf[tg], ouf) < FP64_REL
        assert rel(u[tg], ou) < FP64_REL
