"""The paper's geometric samplers (distance, nearest neighbours) on the GPU
against the oracle, node by node from the same columns: rows exact wherever
the selection cut is clear (the GPU features are float32) and otherwise a
selection within the cut's slack, skeletons and P where the pivots are clear
and otherwise a valid pivoted QR, the far field against the oracle's
evaluation of the GPU's skeletons; the fallback sends nodes to uniform rows
exactly as the oracle decides."""
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
from oracle.skeleton import skeletonize_node
from tests._parity import FP64_REL, check_node_fp64, gkernel, gpu_skeletons, okernel, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def oracle_keys(kind, pool, F, seed, node):
    """The oracle's selection keys of the pool entries (smallest chosen)."""
    P = len(pool)
    if kind == H.DISTANCE:
        return np.array([-math.log(pr.unit_uniform(seed, node | pr.STREAM_KEYS, i)) * max(float(F[i, 0]), 1e-12)
                         for i in range(P)])
    return np.asarray(F[:, 2], dtype=np.float64)


def cut_gap(kind, pool, F, s, seed, node):
    """Relative gap at the selection cut (between the s-th and (s+1)-th smallest oracle keys)."""
    P = len(pool)
    if s >= P:
        return math.inf
    keys = np.sort(oracle_keys(kind, pool, F, seed, node))
    return (keys[s] - keys[s - 1]) / max(abs(keys[s]), 1e-300)


@pytest.mark.parametrize("kind", [H.DISTANCE, H.NEAREST])
def test_heuristic_skeletonize_matches_oracle(ffc, kind):
    X = W.gaussian_mixture(2500, 5, k=8, box=6.0, std=0.5, seed=2)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 160)
    ot = o_build_tree(X, 160)
    sampler = {H.DISTANCE: ffc.SAMPLE_DISTANCE, H.NEAREST: ffc.SAMPLE_NEAREST}[kind]
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=24, num_samples=48, seed=4, sampler=sampler)
    Xt = X[ot.perm]
    # Every node against the oracle's node from the same columns: rows exact where the selection cut is clear
    # (the GPU features are float32), else every chosen key within a 1e-4 slack of the cut; the ID on the GPU's
    # rows as in the plain method.
    kinds = {"exact": 0, "valid": 0}
    cut_exact = 0
    for a in range(1, ot.num_nodes):
        g = sk.node(a)
        cols = g["cols"].astype(np.int64)
        if len(cols) == 0:
            continue
        rows, pool, F = H.heuristic_rows(Xt, ot, a, cols, 48, 4, kind)
        if cut_gap(kind, pool, F, 48, 4, a) >= 1e-4:
            np.testing.assert_array_equal(g["rows"], rows, err_msg=f"{kind} node {a}")
            cut_exact += 1
        else:
            keys = dict(zip(pool.tolist(), oracle_keys(kind, pool, F, 4, a)))
            cut = np.sort(list(keys.values()))[len(rows) - 1]
            assert len(g["rows"]) == len(rows)
            assert all(keys[int(x)] <= cut + 1e-4 * abs(cut) for x in g["rows"]), a
        o = skeletonize_node(Xt, ot, a, cols, ok, 1e-6, 24, 48, 4, rows=g["rows"].astype(np.int64))
        kinds[check_node_fp64(g, o, Xt, ok, 1e-6, 24)] += 1
    print(f"{kind}: {cut_exact} nodes with a clear cut, ID checks {kinds}")
    assert cut_exact >= (ot.num_nodes - 1) // 2
    q = W.charges(ot.N, seed=1)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    ou, ouf = o_evaluate(X, ot, gpu_skeletons(sk, ot.num_nodes), ok, q)
    assert rel(uf.cpu().numpy(), ouf) < FP64_REL
    assert rel(u.cpu().numpy(), ou) < FP64_REL


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
