"""A whole step (skeletonize with reuse + evaluate) captured as a HIP graph and
replayed: every replay must reproduce the eager result exactly, with eager
work (including a skeletonization with another seed that rewrites the same
buffers) between replays."""
import numpy as np
import pytest
import torch

from oracle.kernels import GAUSSIAN, POLYNOMIAL
from paper_1409_2802_amd import workloads as W
from tests._parity import gkernel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


# Mixed precision (2) with the Gaussian on these clusters centres every tile while staging; the
# polynomial kernel takes the split coordinates as they are.
@pytest.mark.parametrize("kind,kw,precision", [(GAUSSIAN, dict(h=1.0), 0), (POLYNOMIAL, dict(h=2.0, p=2), 2),
                                               (GAUSSIAN, dict(h=1.0), 2)])
def test_step_graph_replays_match_eager(ffc, kind, kw, precision):
    X = W.gaussian_mixture(4096, 8, k=8, box=6.0, std=0.5, seed=3)
    q = torch.as_tensor(W.charges(4096, seed=1), device="cuda")
    k = gkernel(kind, **kw)
    opts = dict(tol=1e-7, max_rank=48, num_samples=96, precision=precision, seed=5)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tree = ffc.build_tree(X, 256)
        sk = ffc.skeletonize(tree, k, **opts)
        u_e, uf_e = ffc.evaluate_sum(tree, sk, k, q, precision=precision)
        stream.synchronize()
        u_e, uf_e = u_e.cpu().numpy(), uf_e.cpu().numpy()
        ranks = [sk.node(a)["rank"] for a in range(1, tree.num_nodes)]
        u = torch.zeros(4096, dtype=torch.float64, device="cuda")
        uf = torch.zeros(4096, dtype=torch.float64, device="cuda")
        g = ffc.StepGraph(tree, sk, k, q, u, uf, stream, **opts)
        for rep in range(3):
            # Eager work between replays: a skeletonization with another seed
            # rewrites the shared buffers, and an unrelated direct sum.
            ffc.skeletonize(tree, k, **dict(opts, seed=11 + rep), reuse=sk)
            ffc.direct_sum(X[:64], X, q, k)
            u.zero_()
            uf.zero_()
            g.launch(stream)
            stream.synchronize()
            np.testing.assert_array_equal(u.cpu().numpy(), u_e, err_msg=f"replay {rep}")
            np.testing.assert_array_equal(uf.cpu().numpy(), uf_e, err_msg=f"replay {rep}")
            assert [sk.node(a)["rank"] for a in range(1, tree.num_nodes)] == ranks
        ffc.check_device(stream)


def test_step_graph_rejects_null_stream_and_fallback(ffc):
    X = W.uniform_cube(1024, 4, seed=0)
    q = torch.as_tensor(W.charges(1024, seed=1), device="cuda")
    k = gkernel(GAUSSIAN, h=0.5)
    tree = ffc.build_tree(X, 128)
    sk = ffc.skeletonize(tree, k, tol=1e-6, max_rank=32)
    u = torch.empty(1024, dtype=torch.float64, device="cuda")
    with pytest.raises(ffc.FfcError) as e:
        ffc.StepGraph(tree, sk, k, q, u, None, torch.cuda.default_stream(), tol=1e-6, max_rank=32)
    assert e.value.code == ffc.FFC_ERR_INVALID_ARG


def test_mixed_graph_needs_its_operands_prepared_eagerly(ffc):
    """The matrix-core operands of a tree are prepared by the first eager
    mixed-precision call; capturing before that is refused with FFC_ERR_STATE
    instead of recording a preparation that would only run at replay."""
    X = W.gaussian_mixture(2048, 8, k=4, box=6.0, std=0.5, seed=2)
    q = torch.as_tensor(W.charges(2048, seed=1), device="cuda")
    k = gkernel(GAUSSIAN, h=1.0)
    opts = dict(tol=1e-6, max_rank=32, num_samples=64, seed=1)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tree = ffc.build_tree(X, 256)
        sk = ffc.skeletonize(tree, k, **opts)
        u = torch.zeros(2048, dtype=torch.float64, device="cuda")
        uf = torch.zeros(2048, dtype=torch.float64, device="cuda")
        with pytest.raises(ffc.FfcError) as e:
            ffc.StepGraph(tree, sk, k, q, u, uf, stream, precision=ffc.MIXED_BF16X3, **opts)
        assert e.value.code == ffc.FFC_ERR_STATE
        sk = ffc.skeletonize(tree, k, precision=ffc.MIXED_BF16X3, **opts)
        u_e, uf_e = ffc.evaluate_sum(tree, sk, k, q, precision=ffc.MIXED_BF16X3)
        g = ffc.StepGraph(tree, sk, k, q, u, uf, stream, precision=ffc.MIXED_BF16X3, **opts)
        g.launch(stream)
        stream.synchronize()
        np.testing.assert_array_equal(u.cpu().numpy(), u_e.cpu().numpy())
        np.testing.assert_array_equal(uf.cpu().numpy(), uf_e.cpu().numpy())
    ffc.check_device(stream)


def test_step_graph_replays_match_the_oracle(ffc):
    """Replays of an FP64 step against the oracle's skeletonize + evaluate with the same seed (not only
    against the library's own eager call)."""
    from oracle.evaluate import evaluate as o_evaluate
    from oracle.skeleton import skeletonize as o_skeletonize
    from oracle.tree import build_tree as o_build_tree
    from tests._parity import FP64_REL, okernel, rel, unambiguous
    X = W.gaussian_mixture(4096, 8, k=8, box=6.0, std=0.5, seed=3)
    qh = W.charges(4096, seed=1)
    q = torch.as_tensor(qh, device="cuda")
    k, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    opts = dict(tol=1e-7, max_rank=48, num_samples=96, seed=5)
    ot = o_build_tree(X, 256)
    osk = o_skeletonize(X, ot, ok, 1e-7, 48, 96, seed=5)
    assert all(unambiguous(osk.nodes[a], 1e-7) for a in range(1, ot.num_nodes))
    ou, ouf = o_evaluate(X, ot, osk, ok, qh)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tree = ffc.build_tree(X, 256)
        sk = ffc.skeletonize(tree, k, **opts)
        u = torch.zeros(4096, dtype=torch.float64, device="cuda")
        uf = torch.zeros(4096, dtype=torch.float64, device="cuda")
        g = ffc.StepGraph(tree, sk, k, q, u, uf, stream, **opts)
        for rep in range(2):
            ffc.skeletonize(tree, k, **dict(opts, seed=20 + rep), reuse=sk)
            g.launch(stream)
            stream.synchronize()
            assert rel(u.cpu().numpy(), ou) <= FP64_REL, rep
            assert rel(uf.cpu().numpy(), ouf) <= FP64_REL, rep
            for a in range(1, ot.num_nodes):
                np.testing.assert_array_equal(sk.node(a)["skel"], osk.nodes[a].skel)
    ffc.check_device(stream)


def test_graph_pins_its_buffers_and_defers_frees(ffc):
    """While a step graph holds a skeleton set, calls that would reallocate its buffers (FMM lists for
    another separation, the learned sampler's scratch) fail with FFC_ERR_STATE and change nothing the
    graph reads; freeing the set or the tree only marks it, and the graph keeps replaying the same bits
    until it is freed itself."""
    from oracle.kernels import LAPLACE
    X = W.normal(4096, 3, seed=4)
    q = torch.as_tensor(W.charges(4096, seed=1), device="cuda")
    k = gkernel(LAPLACE)
    opts = dict(tol=1e-6, max_rank=32, num_samples=64, seed=2, separation=1.0)
    lib = ffc.load_library()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tree = ffc.build_tree(X, 128)
        sk = ffc.skeletonize(tree, k, **opts)
        u_e, uf_e = ffc.evaluate_fmm(tree, sk, k, q)
        u_e, uf_e = u_e.cpu().numpy(), uf_e.cpu().numpy()
        u = torch.zeros(4096, dtype=torch.float64, device="cuda")
        uf = torch.zeros(4096, dtype=torch.float64, device="cuda")
        g = ffc.StepGraph(tree, sk, k, q, u, uf, stream, fmm=True, **opts)
        # The same buffer sizes: allowed (the bitmaps and skeletons are rewritten in place).
        ffc.skeletonize(tree, k, **dict(opts, separation=2.0), reuse=sk)
        # New FMM lists would replace buffers the graph reads: refused.
        with pytest.raises(ffc.FfcError) as e:
            ffc.evaluate_fmm(tree, sk, k, q)
        assert e.value.code == ffc.FFC_ERR_STATE and "graph" in str(e.value)
        # The learned sampler's scratch is allocated on first use: refused too.
        prop = ffc.Proposal(W.mlp_init(0))
        with pytest.raises(ffc.FfcError) as e:
            ffc.skeletonize(tree, k, **dict(opts, separation=0.0), proposal=prop, reuse=sk)
        assert e.value.code in (ffc.FFC_ERR_STATE, ffc.FFC_ERR_INVALID_ARG)
        g.launch(stream)
        stream.synchronize()
        np.testing.assert_array_equal(u.cpu().numpy(), u_e)
        np.testing.assert_array_equal(uf.cpu().numpy(), uf_e)
        # Free both handles under the graph: only marked, the graph still replays the same bits.
        lib.ffc_free_skel(sk.handle)
        sk._h = None
        lib.ffc_free_tree(tree.handle)
        tree._h = None
        u.zero_()
        g.launch(stream)
        stream.synchronize()
        np.testing.assert_array_equal(u.cpu().numpy(), u_e)
        g._release()          # the last graph: deletes the marked set and tree
    ffc.check_device(stream)
