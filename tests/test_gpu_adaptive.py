"""Adaptive sample count on the GPU against the oracle: the final row count and
rows of every node bit-exact, skeletons and P where the oracle's pivots and
doubling decisions are clear; the infinite-threshold limit equals plain
skeletonization bitwise; option validation and the refusal to capture it."""
import numpy as np
import pytest
import torch

from oracle.adaptive import skeletonize_adaptive
from oracle.kernels import GAUSSIAN
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from tests._parity import gkernel, okernel, unambiguous

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def clear_decisions(hist, tol_a, margin=1e-6):
    """No held-out error of the node lies within a relative margin of the threshold."""
    return all(abs(err - tol_a) > margin * tol_a for _, err in hist)


@pytest.mark.parametrize("n,d,leaf,s0,tol_a,cap", [(2048, 6, 256, 32, 3e-3, 300), (4096, 8, 512, 48, 1e-3, 400)])
def test_adaptive_matches_oracle(ffc, n, d, leaf, s0, tol_a, cap):
    X = W.gaussian_mixture(n, d, k=8, box=5.0, std=0.6, seed=2)
    gk, ok = gkernel(GAUSSIAN, h=0.6), okernel(GAUSSIAN, h=0.6)
    t = ffc.build_tree(X, leaf)
    sk = ffc.skeletonize(t, gk, tol=1e-7, max_rank=48, num_samples=s0, seed=1, adaptive_tol=tol_a,
                         max_samples=cap)
    ot = o_build_tree(X, leaf)
    osk, hist = skeletonize_adaptive(X, ot, ok, tol=1e-7, max_rank=48, num_samples=s0, seed=1, adaptive_tol=tol_a,
                                     max_samples=cap)
    compared, stop, redos = 0, None, 0
    for level in range(ot.depth, 0, -1):
        for a in ot.level_nodes(level):
            if stop is not None:
                break
            o, g = osk.nodes[a], sk.node(a)
            np.testing.assert_array_equal(g["cols"], o.cols)
            if not clear_decisions(hist[a], tol_a):
                stop = a        # a borderline doubling decision may change everything above it
                break
            np.testing.assert_array_equal(g["rows"], o.rows, err_msg=f"node {a}")
            redos += len(hist[a]) - 1
            if not unambiguous(o, 1e-7):
                stop = a
                break
            assert g["rank"] == o.rank
            np.testing.assert_array_equal(g["skel"], o.skel)
            np.testing.assert_allclose(g["P"], o.P, atol=1e-8 * max(1.0, np.abs(o.P).max()))
            compared += 1
    assert compared >= (1 << ot.depth), (compared, stop)
    assert max(len(h) for h in hist.values()) > 1          # some nodes doubled
    st = sk.stats()
    if stop is None:
        assert st["resampled"] == redos
        assert st["rows_max"] == max(len(o.rows) for o in osk.nodes.values())


def test_infinite_threshold_equals_plain(ffc):
    X = W.gaussian_mixture(4096, 8, k=8, box=5.0, std=0.6, seed=4)
    gk = gkernel(GAUSSIAN, h=0.7)
    t = ffc.build_tree(X, 256)
    a = ffc.skeletonize(t, gk, tol=1e-7, max_rank=40, num_samples=64, seed=2)
    b = ffc.skeletonize(t, gk, tol=1e-7, max_rank=40, num_samples=64, seed=2, adaptive_tol=1e300, max_samples=256)
    for node in range(1, t.num_nodes):
        x, y = a.node(node), b.node(node)
        for key in ("rows", "cols", "skel", "P"):
            np.testing.assert_array_equal(x[key], y[key])
    assert b.stats()["resampled"] == 0


def test_adaptive_option_validation(ffc):
    X = W.uniform_cube(1024, 4, seed=0)
    t = ffc.build_tree(X, 128)
    gk = gkernel(GAUSSIAN, h=0.5)
    for kw, msg in ((dict(adaptive_tol=float("nan")), "finite"),
                    (dict(adaptive_tol=1e-3, max_samples=16), "max_samples"),
                    (dict(adaptive_tol=1e-3, max_samples=-1), "max_samples"),
                    (dict(adaptive_tol=1e-3, max_samples=20000), "8192")):
        with pytest.raises(ffc.FfcError) as e:
            ffc.skeletonize(t, gk, tol=1e-6, max_rank=16, num_samples=32, **kw)
        assert e.value.code == ffc.FFC_ERR_INVALID_ARG and msg in str(e.value)
    # Needs the uniform sampler, and cannot be captured into a graph.
    p = ffc.Proposal(W.mlp_init(0))
    with pytest.raises(ffc.FfcError) as e:
        ffc.skeletonize(t, gk, tol=1e-6, max_rank=16, num_samples=32, proposal=p, adaptive_tol=1e-3)
    assert "uniform sampler" in str(e.value)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=16, num_samples=32, adaptive_tol=1e-3)
    q = torch.as_tensor(W.charges(1024, seed=1), device="cuda")
    u = torch.empty(1024, dtype=torch.float64, device="cuda")
    opts = ffc.SkelOptsC(tol=1e-6, max_rank=16, num_samples=32, precision=0, sampler=0, seed=0, proposal=None,
                         fallback_tol=0.0, pool_factor=0, adaptive_tol=1e-3, max_samples=0)
    import ctypes
    h = ctypes.c_void_p()
    stream = torch.cuda.Stream()
    k = gk.c_struct()
    code = ffc.load_library().ffc_step_graph_create(t.handle, sk.handle, ctypes.byref(k), ctypes.byref(opts),
                                                    ffc._ptr(q), ffc._ptr(u), None, 0,
                                                    ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
    assert code == ffc.FFC_ERR_INVALID_ARG
    assert b"adaptive" in ffc.load_library().ffc_last_error()
