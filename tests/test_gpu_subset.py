"""Skeletonizing a subset of the nodes through the C ABI (node_ids of
ffc_skeletonize_nodes): listed nodes match the oracle, with an internal node's
columns taken from its children's skeletons as the handle holds them; unlisted
nodes keep their bits; bad lists are refused."""
import numpy as np
import pytest
import torch

from oracle.kernels import GAUSSIAN, LAPLACE
from oracle.separation import separated_rows
from oracle.skeleton import skeletonize as o_skeletonize
from oracle.skeleton import skeletonize_node
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from tests._parity import FP64_REL, gkernel, okernel, rel, unambiguous

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def same_node(g, o, tol):
    """The GPU node equals the oracle's: rows exactly, then the skeleton and P where the pivots are clear,
    else a reconstruction no worse than the oracle's on the same block."""
    np.testing.assert_array_equal(g["rows"], o.rows)
    np.testing.assert_array_equal(g["cols"], o.cols)
    if unambiguous(o, tol):
        np.testing.assert_array_equal(g["skel"], o.skel)
        assert rel(g["P"], o.P) <= 1e-8 * max(1.0, np.abs(o.P).max())


def test_subtree_subset_equals_the_full_call(ffc):
    X = W.gaussian_mixture(4096, 6, k=8, box=6.0, std=0.6, seed=2)
    k, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 256)                  # depth 4, nodes 0..30
    ot = o_build_tree(X, 256)
    osk = o_skeletonize(X, ot, ok, 1e-7, 32, 64, seed=3)
    # Node 2's whole subtree plus two leaves elsewhere.
    sub = [2, 5, 6, 11, 12, 13, 14, 23, 24, 25, 26, 27, 28, 29, 30, 15, 18]
    sk = ffc.skeletonize(t, k, tol=1e-7, max_rank=32, num_samples=64, seed=3, node_ids=sub)
    for a in range(1, t.num_nodes):
        g = sk.node(a)
        if a in sub:
            same_node(g, osk.nodes[a], 1e-7)
        else:
            assert g["rank"] == 0 and len(g["cols"]) == 0, a
    ffc.check_device()


@pytest.mark.parametrize("xi", [0.0, 1.0])
def test_subset_redo_on_a_reused_handle(ffc, xi):
    """Full skeletonization with seed 0, then a few nodes (internal and leaves) again with seed 1: each listed
    node equals the oracle's skeletonization of that node from its children's seed-0 skeletons with seed-1
    rows; every other node is bit-identical to before."""
    kind = LAPLACE if xi > 0 else GAUSSIAN
    kw = {} if xi > 0 else dict(h=1.0)
    X = W.gaussian_mixture(4096, 4, k=6, box=5.0, std=0.7, seed=5)
    k, ok = gkernel(kind, **kw), okernel(kind, **kw)
    t = ffc.build_tree(X, 256)
    ot = o_build_tree(X, 256)
    Xt = X[ot.perm]
    opts = dict(tol=1e-7, max_rank=24, num_samples=64, separation=xi)
    sk = ffc.skeletonize(t, k, seed=0, **opts)
    before = {a: sk.node(a) for a in range(1, t.num_nodes)}
    sub = [1, 4, 9, 20, 16]
    ffc.skeletonize(t, k, seed=1, reuse=sk, node_ids=sub, **opts)
    now = {a: sk.node(a) for a in range(1, t.num_nodes)}
    for a in range(1, t.num_nodes):
        if a in sub:
            continue
        for f in ("rank", "cols", "rows", "skel", "P"):
            np.testing.assert_array_equal(now[a][f], before[a][f], err_msg=f"node {a} {f}")
    for a in sorted(sub, reverse=True):          # deepest first, as the library does
        lev = int(np.log2(a + 1))
        if lev == ot.depth:
            cols = np.arange(ot.begin[a], ot.end[a], dtype=np.int64)
        else:
            cols = np.concatenate([now[2 * a + 1]["skel"], now[2 * a + 2]["skel"]]).astype(np.int64)
        rows = separated_rows(Xt, ot, a, 64, 1, xi) if xi > 0 else None
        o = skeletonize_node(Xt, ot, a, cols, ok, 1e-7, 24, 64, 1, rows=rows)
        same_node(now[a], o, 1e-7)
    ffc.check_device()


def test_bad_node_lists_are_refused(ffc):
    X = W.uniform_cube(1024, 3, seed=0)
    t = ffc.build_tree(X, 128)
    k = gkernel(GAUSSIAN, h=0.5)
    for ids in ([0], [t.num_nodes], [3, 3], [-1]):
        with pytest.raises(ffc.FfcError) as e:
            ffc.skeletonize(t, k, tol=1e-6, max_rank=8, node_ids=ids)
        assert e.value.code == ffc.FFC_ERR_INVALID_ARG, ids
    with pytest.raises(ffc.FfcError) as e:
        ffc.skeletonize(t, k, tol=1e-6, max_rank=8, node_ids=[3], adaptive_tol=1e-2)
    assert e.value.code == ffc.FFC_ERR_INVALID_ARG
