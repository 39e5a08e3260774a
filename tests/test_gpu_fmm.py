"""FMM-style evaluation on the GPU against the oracle: every node's skeleton
and far set match (so the interaction lists are the same), u and the far
field to the FP64 bar, FP32 within 1e-4; an infinite separation
giving the direct sum; cached lists rebuilt when the separation changes;
errors for a skeleton set without separation and for the mixed precision."""
import numpy as np
import pytest
import torch

from oracle import fmm as F
from oracle import separation as S
from oracle.direct import direct_sum
from oracle.kernels import GAUSSIAN, LAPLACE, POLYNOMIAL
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


def clear_far_set(Xt, ot, a, xi, margin=1e-9):
    b, e = int(ot.begin[a]), int(ot.end[a])
    diff = Xt - ot.centroid[a]
    d2 = np.einsum("ij,ij->i", diff, diff)
    thr2 = (xi * ot.radius[a]) ** 2
    out = np.r_[0:b, e:ot.N]
    return bool(np.all(np.abs(d2[out] - thr2) > margin * max(thr2, 1e-300)))


CASES = [
    (GAUSSIAN, dict(h=1.0), 1.0, 3000, 3, 100),
    (LAPLACE, dict(), 1.0, 3000, 3, 100),
    (LAPLACE, dict(), 0.8, 2500, 4, 160),
    (POLYNOMIAL, dict(h=4.0, p=3), 0.7, 2000, 5, 128),
]


@pytest.mark.parametrize("kind,kw,xi,n,d,leaf", CASES)
def test_fmm_matches_oracle(ffc, kind, kw, xi, n, d, leaf):
    X = W.gaussian_mixture(n, d, k=6, box=5.0, std=0.7, seed=5)
    gk, ok = gkernel(kind, **kw), okernel(kind, **kw)
    t = ffc.build_tree(X, leaf)
    ot = o_build_tree(X, leaf)
    Xt = X[ot.perm]
    sk = ffc.skeletonize(t, gk, tol=1e-7, max_rank=24, num_samples=64, seed=3, separation=xi)
    osk = S.skeletonize_separated(X, ot, ok, 1e-7, 24, 64, 3, xi)
    far, near = F.fmm_lists(Xt, ot, xi)
    assert sum(len(v) for v in far.values()) > 0
    same = all(np.array_equal(sk.node(a)["skel"], osk.nodes[a].skel) and unambiguous(osk.nodes[a], 1e-7)
               and clear_far_set(Xt, ot, a, xi) for a in range(1, ot.num_nodes))
    assert same          # these cases have no near-tie in any pivot, far set or admissibility test
    q = W.charges(ot.N, seed=1)
    u, uf = ffc.evaluate_fmm(t, sk, gk, q)
    ffc.check_device()
    ou, ouf = F.fmm_evaluate(X, ot, osk, ok, q, xi)
    ref = direct_sum(X, X, q, ok)
    # Always: the GPU sum is as accurate as the method allows.
    assert rel(u.cpu().numpy(), ref) < max(10 * rel(ou, ref), 1e-12)
    assert rel(u.cpu().numpy(), ou) < FP64_REL
    assert rel(uf.cpu().numpy(), ouf) < FP64_REL
    u32, _ = ffc.evaluate_fmm(t, sk, gk, q, precision=ffc.FP32)
    assert rel(u32.cpu().numpy(), ou) < 1e-4
    # The lists are cached: a second call gives the same bits.
    u2, _ = ffc.evaluate_fmm(t, sk, gk, q)
    assert torch.equal(u, u2)


def test_fmm_infinite_separation_is_direct_sum(ffc):
    X = W.gaussian_mixture(2100, 4, k=6, box=5.0, std=0.7, seed=6)
    gk, ok = gkernel(GAUSSIAN, h=0.8), okernel(GAUSSIAN, h=0.8)
    t = ffc.build_tree(X, 120)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=16, num_samples=48, seed=2, separation=1e300)
    q = W.charges(2100, seed=3)
    u, uf = ffc.evaluate_fmm(t, sk, gk, q)
    assert torch.count_nonzero(uf).item() == 0
    assert rel(u.cpu().numpy(), direct_sum(X, X, q, ok)) < 1e-12


def test_fmm_lists_follow_the_separation(ffc):
    X = W.gaussian_mixture(3000, 3, k=6, box=5.0, std=0.7, seed=8)
    gk = gkernel(LAPLACE)
    t = ffc.build_tree(X, 100)
    q = W.charges(3000, seed=4)
    kw = dict(tol=1e-7, max_rank=24, num_samples=64, seed=3)
    sk = ffc.skeletonize(t, gk, separation=0.7, **kw)
    ffc.evaluate_fmm(t, sk, gk, q)
    ffc.skeletonize(t, gk, separation=1.3, reuse=sk, **kw)      # same handle, new separation
    u, _ = ffc.evaluate_fmm(t, sk, gk, q)
    fresh = ffc.skeletonize(t, gk, separation=1.3, **kw)
    v, _ = ffc.evaluate_fmm(t, fresh, gk, q)
    assert torch.equal(u, v)


def test_fmm_errors(ffc):
    X = W.uniform_cube(1024, 4, seed=0)
    t = ffc.build_tree(X, 128)
    gk = gkernel(GAUSSIAN, h=0.5)
    q = W.charges(1024, seed=1)
    plain = ffc.skeletonize(t, gk, tol=1e-6, max_rank=16, num_samples=32)
    with pytest.raises(ffc.FfcError) as e:
        ffc.evaluate_fmm(t, plain, gk, q)
    assert e.value.code == ffc.FFC_ERR_STATE
    sep = ffc.skeletonize(t, gk, tol=1e-6, max_rank=16, num_samples=32, separation=1.0)
    with pytest.raises(ffc.FfcError) as e:
        ffc.evaluate_fmm(t, sep, gk, q, precision=ffc.MIXED_BF16X3)
    assert e.value.code == ffc.FFC_ERR_INVALID_ARG


def test_fmm_graph_replays(ffc):
    """A step graph with the FMM-style evaluation: refused before the lists exist and without separation;
    replays give the eager bits, with an eager skeletonization of another seed between them."""
    X = W.gaussian_mixture(4096, 3, k=6, box=5.0, std=0.7, seed=7)
    gk = gkernel(LAPLACE)
    t = ffc.build_tree(X, 128)
    kw = dict(tol=1e-7, max_rank=24, num_samples=64, seed=4, separation=1.0)
    q = torch.as_tensor(W.charges(4096, seed=2), device="cuda")
    u = torch.zeros_like(q)
    uf = torch.zeros_like(q)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sk = ffc.skeletonize(t, gk, **kw)
        with pytest.raises(ffc.FfcError) as e:     # interaction lists not built yet
            ffc.StepGraph(t, sk, gk, q, u, uf, stream, fmm=True, **kw)
        assert e.value.code == ffc.FFC_ERR_STATE
        eager, eager_far = ffc.evaluate_fmm(t, sk, gk, q)
        with pytest.raises(ffc.FfcError) as e:
            ffc.StepGraph(t, sk, gk, q, u, uf, stream, fmm=True, **dict(kw, separation=0.0))
        assert e.value.code == ffc.FFC_ERR_INVALID_ARG
        g = ffc.StepGraph(t, sk, gk, q, u, uf, stream, fmm=True, **kw)
        for rep in range(3):
            ffc.skeletonize(t, gk, **dict(kw, seed=11 + rep), reuse=sk)
            u.zero_()
            uf.zero_()
            g.launch(stream)
            stream.synchronize()
            assert torch.equal(u, eager) and torch.equal(uf, eager_far), rep
    ffc.check_device(stream)
