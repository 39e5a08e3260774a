"""GPU ball tree and row sampler against the oracle (Section 2 tree groupings;
Section 4.1.3 uniform sampling without replacement). Both are index work and
must agree bit for bit."""
import numpy as np
import pytest
import torch

from oracle.sampling import sample_far_rows
from oracle.tree import build_partition as o_partition
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from tests._parity import gkernel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


CASES = [
    ("uniform", lambda: W.uniform_cube(2048, 4, seed=0), 256),
    ("mixture", lambda: W.gaussian_mixture(5000, 16, k=8, box=10.0, std=0.5, seed=1), 100),
    ("subspace", lambda: W.low_intrinsic(3001, 64, di=8, noise=1e-2, seed=2), 128),
    ("highdim", lambda: W.highdim_clusters(1500, 1000, k=16, seed=3), 200),
    ("tiny", lambda: W.uniform_cube(3, 2, seed=4), 1),
    ("one-dim", lambda: W.uniform_cube(777, 1, seed=5), 50),
    ("single", lambda: W.uniform_cube(1, 3, seed=6), 4),
]


@pytest.mark.parametrize("name,make,leaf", CASES, ids=[c[0] for c in CASES])
def test_tree_matches_oracle(ffc, name, make, leaf):
    X = make()
    t = ffc.build_tree(X, leaf)
    o = o_build_tree(X, leaf)
    a = t.arrays()
    assert t.depth == o.depth
    np.testing.assert_array_equal(a["begin"], o.begin)
    np.testing.assert_array_equal(a["end"], o.end)
    np.testing.assert_array_equal(a["perm"], o.perm)
    np.testing.assert_allclose(a["centroid"], o.centroid, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a["radius"], o.radius, rtol=1e-12, atol=1e-12)


def test_partition_matches_oracle(ffc):
    X = W.uniform_cube(2048, 4, seed=0)
    t = ffc.build_partition(X, 256)
    o = o_partition(X, 256)
    a = t.arrays()
    np.testing.assert_array_equal(a["perm"], np.arange(2048))
    np.testing.assert_array_equal(a["begin"], o.begin)
    np.testing.assert_allclose(a["centroid"], o.centroid, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("N,leaf,s,seed", [(2048, 256, 128, 0), (5000, 100, 60, 7), (700, 64, 1000, 3),
                                           (4096, 512, 512, 11)])
def test_sampled_rows_bit_exact(ffc, N, leaf, s, seed):
    X = W.uniform_cube(N, 3, seed=seed)
    t = ffc.build_tree(X, leaf)
    sk = ffc.skeletonize(t, gkernel(0, h=0.3), tol=1e-3, max_rank=8, num_samples=s, seed=seed)
    a = t.arrays()
    for node in range(1, t.num_nodes):
        got = sk.node(node)["rows"]
        want = sample_far_rows(int(a["begin"][node]), int(a["end"][node]), N, s, seed, node)
        np.testing.assert_array_equal(got, want)
