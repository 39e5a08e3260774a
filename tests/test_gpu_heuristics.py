"""The paper's geometric samplers (distance, nearest neighbours) on the GPU
against the oracle: rows exact wherever the selection cut is clear (the GPU
features are float32), skeletons and P where the pivots are clear, far field
to the FP64 bar when every node matched; the fallback sends nodes to uniform
rows exactly as the oracle decides."""
import math

import numpy as np
import pytest
import torch

from oracle import heuristics as H
from oracle import proposal as pr
from oracle.evaluate import evaluate as o_evaluate
from oracle.kernels import GAUSSIAN
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


def cut_gap(kind, pool, F, s, seed, node):
    """Relative gap at the selection cut (between the s-th and (s+1)-th smallest oracle keys)."""
    P = len(pool)
    if s >= P:
        return math.inf
    if kind == H.DISTANCE:
        keys = [-math.log(pr.unit_uniform(seed, node | pr.STREAM_KEYS, i)) * max(float(F[i, 0]), 1e-12)
                for i in range(P)]
    else:
        keys = list(F[:, 2])
    keys = np.sort(keys)
    return (keys[s] - keys[s - 1]) / max(abs(keys[s]), 1e-300)


@pytest.mark.parametrize("kind", [H.DISTANCE, H.NEAREST])
def test_heuristic_skeletonize_matches_oracle(ffc, kind):
    X = W.gaussian_mixture(2500, 5, k=8, box=6.0, std=0.5, seed=2)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 160)
    ot = o_build_tree(X, 160)
    sampler = {H.DISTANCE: ffc.SAMPLE_DISTANCE, H.NEAREST: ffc.SAMPLE_NEAREST}[kind]
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=24, num_samples=48, seed=4, sampler=sampler)
    osk, fell = H.skeletonize_heuristic(X, ot, ok, 1e-6, 24, 48, 4, kind)
    Xt = X[ot.perm]
    exact, checked = 0, 0
    for level in range(ot.depth, 0, -1):
        for a in ot.level_nodes(level):
            g, o = sk.node(a), osk.nodes[a]
            if not np.array_equal(g["cols"], o.cols):
                continue                            # an ambiguous choice below changed the columns
            checked += 1
            if len(o.cols) == 0:
                continue
            _, pool, F = H.heuristic_rows(Xt, ot, a, o.cols, 48, 4, kind)
            if cut_gap(kind, pool, F, 48, 4, a) < 1e-4:
                continue
            np.testing.assert_array_equal(g["rows"], o.rows, err_msg=f"{kind} node {a}")
            if not unambiguous(o, 1e-6):
                continue
            assert g["rank"] == o.rank, f"node {a}"
            np.testing.assert_array_equal(g["skel"], o.skel)
            np.testing.assert_allclose(g["P"], o.P, atol=1e-8 * max(1.0, np.abs(o.P).max()))
            exact += 1
    assert checked == ot.num_nodes - 1
    assert exact >= 0.8 * checked, (exact, checked)
    q = W.charges(ot.N, seed=1)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    ou, ouf = o_evaluate(X, ot, osk, ok, q)
    if exact == checked:
        assert rel(uf.cpu().numpy(), ouf) < FP64_REL


@pytest.mark.parametrize("sampler_name", ["SAMPLE_DISTANCE", "SAMPLE_NEAREST"])
def test_heuristic_fallback_to_uniform(ffc, sampler_name):
    X = W.gaussian_mixture(2500, 5, k=8, box=6.0, std=0.5, seed=2)
    gk = gkernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 160)
    sampler = getattr(ffc, sampler_name)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=24, num_samples=48, seed=4, sampler=sampler,
                         fallback_tol=1e-300)
    uni = ffc.skeletonize(t, gk, tol=1e-6, max_rank=24, num_samples=48, seed=4)
    leaves = range((1 << t.depth) - 1, t.num_nodes)
    fallen = [a for a in leaves if np.array_equal(sk.node(a)["rows"], uni.node(a)["rows"])]
    assert len(fallen) >= len(leaves) // 2
    assert sk.stats()["fallbacks"] >= len(fallen)
    keep = ffc.skeletonize(t, gk, tol=1e-6, max_rank=24, num_samples=48, seed=4, sampler=sampler,
                           fallback_tol=1e300)
    assert keep.stats()["fallbacks"] == 0
