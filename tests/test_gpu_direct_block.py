"""GPU direct sum and sampled kernel blocks against the oracle (Section 1,
eq. e:sum; Section 2.2, the sampled block K')."""
import numpy as np
import pytest
import torch

from oracle.direct import direct_abs_sum, direct_sum as o_direct
from oracle.kernels import kernel_matrix
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from tests._parity import KERNELS, direct_bound, gkernel, okernel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def test_laplace_d3_coincident_and_tiny_distances(ffc):
    """The d = 3 Laplace kernel (1/r, its own kernel instances): coincident points give 0, and squared
    distances in (0, 2^-900], below the range of the reciprocal square root estimate, take the general
    power; both in the direct sum against the oracle."""
    Y = W.normal(70, 3, seed=4)
    X = W.normal(130, 3, seed=5)
    X[:3] = Y[:3]                              # r = 0
    Y[3:6] = 0.0
    X[3:6] = 0.0
    X[3:6, 0] = [1e-140, 3e-137, 2e-160]       # r^2 = 1e-280, 9e-274, 4e-320 (subnormal)
    q = W.charges(130, seed=6)
    k = dict()
    u = ffc.direct_sum(Y, X, q, gkernel(1, **k)).cpu().numpy()
    ref = o_direct(Y, X, q, okernel(1, **k))
    assert np.all(np.isfinite(u)) and np.abs(u[3:6]).min() > 1e130
    assert np.all(np.abs(u - ref) <= direct_bound(Y, X, q, 1, k))
    ffc.check_device()


@pytest.mark.parametrize("name", list(KERNELS))
@pytest.mark.parametrize("m,n,d", [(1, 1, 3), (65, 130, 4), (333, 1000, 16), (200, 257, 64), (70, 90, 1000)])
def test_direct_sum_fp64(ffc, name, m, n, d):
    kind, kw = KERNELS[name]
    if kind == 1 and d < 3:
        pytest.skip("Laplace needs d >= 3")
    Y = W.normal(m, d, seed=1) / np.sqrt(d)
    X = W.normal(n, d, seed=2) / np.sqrt(d)
    if m >= 3 and n >= 3:
        X[:3] = Y[:3]          # coincident pairs: the Laplace kernel must give 0 there
    q = W.charges(n, seed=3)
    u = ffc.direct_sum(Y, X, q, gkernel(kind, **kw)).cpu().numpy()
    ref = o_direct(Y, X, q, okernel(kind, **kw))
    assert np.all(np.abs(u - ref) <= direct_bound(Y, X, q, kind, kw))
    ffc.check_device()


@pytest.mark.parametrize("name", list(KERNELS))
def test_direct_sum_fp32(ffc, name):
    kind, kw = KERNELS[name]
    Y = W.uniform_cube(300, 8, seed=4)
    X = W.uniform_cube(500, 8, seed=5) + 0.05
    q = W.charges(500, seed=6)
    u = ffc.direct_sum(Y, X, q, gkernel(kind, **kw), precision=ffc.FP32).cpu().numpy()
    ref = o_direct(Y, X, q, okernel(kind, **kw))
    scale = direct_abs_sum(Y, X, q, okernel(kind, **kw))
    # FP32 distances: relative error of each kernel value ~ (d + |log K|) * 2^-23 times the power for Laplace.
    bound = {0: 5e-5, 1: 5e-5, 2: 5e-5}[kind]
    assert np.all(np.abs(u - ref) <= bound * scale)


@pytest.mark.parametrize("name", list(KERNELS))
@pytest.mark.parametrize("N,d,s,n", [(600, 4, 37, 129), (3000, 16, 128, 200), (900, 100, 70, 65)])
def test_sampled_block_fp64(ffc, name, N, d, s, n):
    kind, kw = KERNELS[name]
    X = W.gaussian_mixture(N, d, k=5, box=3.0, std=0.5, seed=7)
    t = ffc.build_tree(X, 64)
    perm = t.arrays()["perm"]
    g = np.random.default_rng(8)
    rows = g.choice(N, size=s, replace=False).astype(np.int32)
    cols = g.choice(N, size=n, replace=False).astype(np.int32)
    Kg = ffc.sampled_block(t, gkernel(kind, **kw), rows, cols).cpu().numpy()
    Xt = X[perm]
    Ko = kernel_matrix(Xt[rows], Xt[cols], okernel(kind, **kw))
    np.testing.assert_allclose(Kg, Ko, rtol=1e-12, atol=0)


def test_nonfinite_kernel_value_sets_the_flag(ffc):
    # d = 7: r^-5 overflows for r = 1e-70 (1e350); the flag is raised once and cleared by the check.
    ffc.check_device()
    X = W.normal(40, 7, seed=8)
    X[0] = 0.0
    X[1] = 0.0
    X[1, 0] = 1e-70
    q = W.charges(40, seed=9)
    k = gkernel(1)
    ffc.direct_sum(X, X, q, k)
    with pytest.raises(ffc.FfcError) as e:
        ffc.check_device()
    assert e.value.code == ffc.FFC_ERR_NONFINITE
    ffc.check_device()
    ffc.direct_sum(X[2:], X[2:], q[2:], k)     # well-separated points: no flag
    ffc.check_device()
