"""Parity at the workloads' full sizes, in the configuration bench.py times.

Every node is checked against the oracle's skeletonization of that node from
the same columns (the GPU's children skeletons), so a near-tie below does not
stop the comparison above it: rows bit-exact; skeleton, rank and P equal where
the oracle's pivots are clear, and otherwise a valid pivoted QR of the same
block (every pivot within a relative 1e-9 of the largest trailing norm, the
rank rule holding) with a reconstruction as good as the oracle's. The kernel
sum is compared with the oracle's evaluation of the GPU's own skeletons at
every target (or sampled targets), so it is checked whatever the ties.
Reduced-precision paths (FP32, mixed) are held to the exact FP64 block: the
GPU's skeleton must reconstruct it to twice the oracle's residual plus the
kernel values' error bound times (1 + |P|_2).

Workloads: mixture16 (N = 65536, d = 16) in FP64 and FP32; the separated
Laplace trees (N = 65536, d = 3; treecode at separation 2, FMM-style at 1);
highdim1000 / highdim1000g (N = 65536, d = 1000) in mixed precision on 64
seeded random nodes; subspace64 (N = 262144, d = 64, Laplace) in mixed
precision on sampled leaves; learned64 (the same points, Gaussian h = 1,
learned proposal, mixed) on sampled nodes, and the same points with 1024
sampled rows (uniform, mixed)."""
import numpy as np
import pytest
import torch

from oracle.direct import direct_sum as o_direct
from oracle.evaluate import evaluate as o_evaluate
from oracle.fmm import fmm_evaluate
from oracle.kernels import GAUSSIAN, LAPLACE, POLYNOMIAL, kernel_matrix
from oracle.separation import separated_rows, treecode_evaluate
from oracle.skeleton import skeletonize_node
from oracle.tree import build_tree as o_build_tree
from paper_1409_2802_amd import workloads as W
from tests._parity import (FP64_REL, check_node_fp64, direct_bound, gkernel, gpu_skeletons, local_pivots, okernel,
                           recon_residual, rel)

pytestmark = pytest.mark.gpu

# Relative error of one kernel value in the reduced-precision modes (bounds of the tile arithmetic):
# FP32 explicit differences carry r^2 to about (d + 2) 2^-24; the mixed Gram split to 2^-15 of
# (|y - c| + |x - c|)^2 (the bound of the mixed direct-sum tests).
U32 = 2.0 ** -24
GRAM_REL = 2.0 ** -15


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def node_cols(g):
    return g["cols"].astype(np.int64)


def check_node_reduced(g, o, Xt, ok, kerr):
    """Reduced-precision node: same rows and columns as the oracle; its skeleton and P reconstruct the exact
    FP64 block to twice the oracle's residual plus kerr (1 + |P|_2)."""
    np.testing.assert_array_equal(g["rows"], o.rows)
    np.testing.assert_array_equal(g["cols"], o.cols)
    A = kernel_matrix(Xt[o.rows], Xt[o.cols], ok)
    J = local_pivots(g)
    np.testing.assert_array_equal(g["P"][:, J], np.eye(g["rank"]))
    r_o = recon_residual(A, o.piv[:o.rank], o.P)
    r_g = recon_residual(A, J, g["P"])
    pn = np.linalg.norm(g["P"], 2) if g["rank"] else 0.0
    assert r_g <= 2 * r_o + kerr * (1 + pn) + 1e-12, (r_g, r_o, kerr, pn)
    return r_g, r_o


def oracle_nodes(jobs, workers=8):
    """Run oracle node computations (callables) on threads: numpy's kernels release the GIL."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda f: f(), jobs))


def gram_kerr_gaussian(Y, X, c, h):
    """Bound on the relative error of Gaussian kernel values from the split Gram, centred on c."""
    span = (np.linalg.norm(Y - c, axis=1).max() + np.linalg.norm(X - c, axis=1).max()) ** 2
    return GRAM_REL * span / (2 * h * h) + 2.0 ** -20


def test_mixture16_every_node(ffc):
    """N=65536, d=16, 32 clusters, Gaussian h=1, leaf 512, s=512, rank cap 256, tol 1e-5, FP64: all 254 nodes,
    and the whole sum at every target against the oracle's evaluation of the same skeletons."""
    X = W.gaussian_mixture(65536, 16, k=32, box=10.0, std=0.5, seed=0)
    q = W.charges(65536, seed=1)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 512)
    sk = ffc.skeletonize(t, gk, tol=1e-5, max_rank=256, num_samples=512, seed=0)
    u, uf = ffc.evaluate_sum(t, sk, gk, q)
    ot = o_build_tree(X, 512)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    Xt = X[ot.perm]
    kinds = {"exact": 0, "valid": 0}
    gnodes = {a: sk.node(a) for a in range(1, ot.num_nodes)}
    onodes = oracle_nodes([lambda a=a: skeletonize_node(Xt, ot, a, node_cols(gnodes[a]), ok, 1e-5, 256, 512, 0)
                           for a in gnodes])
    for (a, g), o in zip(gnodes.items(), onodes):
        kinds[check_node_fp64(g, o, Xt, ok, 1e-5, 256)] += 1
    print("mixture16 nodes:", kinds)
    assert kinds["exact"] >= (1 << ot.depth)
    ou, ouf = o_evaluate(X, ot, gpu_skeletons(sk, ot.num_nodes), ok, q)
    assert rel(uf.cpu().numpy(), ouf) < FP64_REL
    assert rel(u.cpu().numpy(), ou) < FP64_REL


def test_mixture16_fp32(ffc):
    """The FP32 variant of the same step: rows exact; 48 random nodes' skeletons reconstruct the exact FP64 block
    within the FP32 kernel error; the whole sum within 1e-4 of the oracle's FP64 evaluation of the GPU's
    skeletons on 4096 sampled targets (FP32 values summed in FP64)."""
    X = W.gaussian_mixture(65536, 16, k=32, box=10.0, std=0.5, seed=0)
    q = W.charges(65536, seed=1)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 512)
    sk = ffc.skeletonize(t, gk, tol=1e-5, max_rank=256, num_samples=512, seed=0, precision=ffc.FP32)
    u, uf = ffc.evaluate_sum(t, sk, gk, q, precision=ffc.FP32)
    ot = o_build_tree(X, 512)
    Xt = X[ot.perm]
    picks = [int(a) for a in np.random.default_rng(3).choice(np.arange(1, ot.num_nodes), 48, replace=False)]
    gnodes = {a: sk.node(a) for a in picks}
    onodes = oracle_nodes([lambda a=a: skeletonize_node(Xt, ot, a, node_cols(gnodes[a]), ok, 1e-5, 256, 512, 0)
                           for a in picks])
    for a, o in zip(picks, onodes):
        g = gnodes[a]
        # exp of r^2 / 2h^2 with r^2 relative error (d + 2) u32: relative error (d + 2) u32 r^2 / 2h^2 + u32.
        Y, C = Xt[o.rows], Xt[o.cols]
        r2max = float(((Y[:, None, :] - C[None, :, :]) ** 2).sum(-1).max())
        check_node_reduced(g, o, Xt, ok, (16 + 2) * U32 * r2max / 2 + 4 * U32)
    # FP32 kernel values err by at most (d + 2) u32 r^2 / 2h^2 (about 1e-5 at the r^2 <= 16 of in-cluster
    # pairs); sums of random-sign terms can lose another factor 10 to cancellation.
    tg = W.subset(65536, 4096, seed=5)
    ou, ouf = o_evaluate(X, ot, gpu_skeletons(sk, ot.num_nodes), ok, q)
    assert rel(uf.cpu().numpy()[tg], ouf[tg]) < 1e-4
    assert rel(u.cpu().numpy()[tg], ou[tg]) < 1e-4


@pytest.mark.parametrize("kind,kw", [(POLYNOMIAL, dict(h=1.0, p=3)), (GAUSSIAN, dict(h=1.5))])
def test_highdim1000_mixed_64_nodes(ffc, kind, kw):
    """N=65536, d=1000 (N(0,I)/sqrt(d) + 64 offsets of norm 3), leaf 512, s=512, rank cap 256, tol 1e-4, in the
    mixed precision bench.py times (bf16 hi/lo Gram on matrix cores): 64 seeded random nodes against the FP64
    oracle on the same rows and columns; then 48 sampled targets of the FP64 direct sum."""
    N, d = 65536, 1000
    X = W.highdim_clusters(N, d, k=64, seed=0)
    q = W.charges(N, seed=1)
    gk, ok = gkernel(kind, **kw), okernel(kind, **kw)
    t = ffc.build_tree(X, 512)
    sk = ffc.skeletonize(t, gk, tol=1e-4, max_rank=256, num_samples=512, seed=0, precision=ffc.MIXED_BF16X3)
    ffc.check_device()
    ot = o_build_tree(X, 512)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    Xt = X[ot.perm]
    res = []
    picks = [int(a) for a in np.random.default_rng(0).choice(np.arange(1, ot.num_nodes), 64, replace=False)]
    gnodes = {a: sk.node(a) for a in picks}
    onodes = oracle_nodes([lambda a=a: skeletonize_node(Xt, ot, a, node_cols(gnodes[a]), ok, 1e-4, 256, 512, 0)
                           for a in picks])
    for a, o in zip(picks, onodes):
        g = gnodes[a]
        Y, C = Xt[o.rows], Xt[o.cols]
        if kind == GAUSSIAN:
            kerr = gram_kerr_gaussian(Y, C, ot.centroid[a], kw["h"])
        else:   # raw inner products: p |d(x.y)| / |x.y + c| with |d(x.y)| <= GRAM_REL |x||y|
            base = np.abs(Y @ C.T + 1.0)
            kerr = kw["p"] * float((GRAM_REL * np.outer(np.linalg.norm(Y, axis=1), np.linalg.norm(C, axis=1))
                                    / np.maximum(base, 1e-300)).max()) + 2.0 ** -20
        res.append(check_node_reduced(g, o, Xt, ok, kerr))
    r = np.array(res)
    print(f"highdim1000 {kind}: GPU residual mean {r[:, 0].mean():.3e}, oracle {r[:, 1].mean():.3e}")
    tg = W.subset(N, 48, seed=2)
    Xd = torch.as_tensor(X, device="cuda")
    u = ffc.direct_sum(Xd[tg], Xd, q, gk).cpu().numpy()
    uo = o_direct(X[tg], X, q, ok)
    assert np.all(np.abs(u - uo) <= direct_bound(X[tg], X, q, kind, kw))


def test_subspace64_mixed_leaves(ffc):
    """N=262144, d=64 near an 8-dim subspace, Laplace |x-y|^-62, leaf 1024, s=512, rank cap 256, tol 1e-6 in the
    mixed precision bench.py times (three-part split on matrix cores): the tree, and 8 sampled leaves against the
    FP64 oracle on the same rows; the kernel error bound is the power (31) times the r^2 bound of the Laplace
    tiles, (2d + 4) 2^-20."""
    N, d = 262144, 64
    X = W.low_intrinsic(N, d, di=8, noise=1e-2, seed=0)
    gk, ok = gkernel(LAPLACE), okernel(LAPLACE)
    t = ffc.build_tree(X, 1024)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=256, num_samples=512, seed=0, precision=ffc.MIXED_BF16X3)
    ffc.check_device()
    ot = o_build_tree(X, 1024)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    Xt = X[ot.perm]
    kerr = (d - 2) / 2 * (2 * d + 4) * 2.0 ** -20
    picks = [int(a) for a in np.random.default_rng(8).choice(list(ot.level_nodes(ot.depth)), 8, replace=False)]
    gnodes = {a: sk.node(a) for a in picks}
    onodes = oracle_nodes([lambda a=a: skeletonize_node(Xt, ot, a, node_cols(gnodes[a]), ok, 1e-6, 256, 512, 0)
                           for a in picks])
    for a, o in zip(picks, onodes):
        check_node_reduced(gnodes[a], o, Xt, ok, kerr)


def test_learned64_sampled_nodes(ffc):
    """The default bench workload at full size: N=262144, d=64, Gaussian h=1, leaf 1024, s=512, rank cap 256,
    mixed precision, rows from a proposal trained on the GPU (here 64 blocks). On 12 sampled leaves and 2 nodes
    of every other level: the rows are exactly the oracle's selection from the same pool, features and network (or, where the
    s-th and (s+1)-th keys are within 1e-4, a selection whose keys all lie within that slack of the cut), and
    the GPU's skeleton reconstructs the exact FP64 block of those rows within the mixed kernel error."""
    from oracle import proposal as pr
    N, d = 262144, 64
    X = W.low_intrinsic(N, d, di=8, noise=1e-2, seed=0)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 1024)
    p = ffc.Proposal(W.mlp_init(5))
    p.train(t, gk, 64, 512, 4096, epochs=2, batch=4096, lr=1e-3, eps=1e-4, seed=7)
    th, mu, sd = (np.asarray(a, dtype=np.float64) for a in p.get())
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=256, num_samples=512, seed=0, precision=ffc.MIXED_BF16X3,
                         proposal=p, pool_factor=8)
    ffc.check_device()
    ot = o_build_tree(X, 1024)
    Xt = X[ot.perm]
    rng = np.random.default_rng(9)
    picks = []
    for level in range(ot.depth, 0, -1):
        nodes = list(ot.level_nodes(level))
        picks += [int(a) for a in rng.choice(nodes, min(len(nodes), 12 if level == ot.depth else 2), replace=False)]
    gnodes = {a: sk.node(a) for a in picks}

    def oracle_side(a):
        g = gnodes[a]
        cols = node_cols(g)
        b, e = int(ot.begin[a]), int(ot.end[a])
        pool = pr.candidate_pool(b, e, ot.N, 512, 0, a, 8)
        sc, _ = pr.mlp_forward(th, pr.standardize(pr.features(Xt[pool], pr.column_geometry(Xt[cols], 0, a)), mu, sd))
        o, _ = pr.skeletonize_learned_node(Xt, ot, a, cols, ok, 1e-6, 256, 512, 0, th, mu, sd, 0.0, 8)
        o_rows = skeletonize_node(Xt, ot, a, cols, ok, 1e-6, 256, 512, 0, rows=g["rows"].astype(np.int64))
        return pool, sc, o, o_rows

    exact = 0
    for a, (pool, sc, o, o_rows) in zip(picks, oracle_nodes([lambda a=a: oracle_side(a) for a in picks])):
        g = gnodes[a]
        if np.array_equal(g["rows"], o.rows):
            exact += 1
        else:
            # The GPU's rows against the oracle's keys: each chosen key within the cut plus a 1e-4 slack
            # (float32 scores move keys near the cut), and as many rows as the oracle chose.
            keys = dict(zip(pool.tolist(), pr.selection_keys(sc, 0, a)))
            assert len(g["rows"]) == len(o.rows)
            cut = sorted(keys.values())[len(o.rows) - 1]
            assert all(keys[int(x)] <= cut * (1 + 1e-4) for x in g["rows"]), a
        kerr = gram_kerr_gaussian(Xt[g["rows"]], Xt[node_cols(g)], ot.centroid[a], 1.0)
        check_node_reduced(g, o_rows, Xt, ok, kerr)
    assert exact >= 10
    print("learned64 sampled nodes with the oracle's exact rows:", exact)


def test_learned64_points_1024_rows(ffc):
    """The learned64 points with 1024 sampled rows per node (4x the rank cap, the register-resident QR's 32-lane
    groups): N=262144, d=64, Gaussian h=1, leaf 1024, rank cap 256, uniform rows, mixed precision. On 4 sampled
    leaves and 1 node of every other level the rows equal the oracle's, and the GPU's skeleton reconstructs the
    exact FP64 block of those rows within the mixed kernel error."""
    N, d = 262144, 64
    X = W.low_intrinsic(N, d, di=8, noise=1e-2, seed=0)
    gk, ok = gkernel(GAUSSIAN, h=1.0), okernel(GAUSSIAN, h=1.0)
    t = ffc.build_tree(X, 1024)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=256, num_samples=1024, seed=0, precision=ffc.MIXED_BF16X3)
    ffc.check_device()
    ot = o_build_tree(X, 1024)
    Xt = X[ot.perm]
    rng = np.random.default_rng(10)
    picks = []
    for level in range(ot.depth, 0, -1):
        nodes = list(ot.level_nodes(level))
        picks += [int(a) for a in rng.choice(nodes, 4 if level == ot.depth else 1, replace=False)]
    gnodes = {a: sk.node(a) for a in picks}
    onodes = oracle_nodes([lambda a=a: skeletonize_node(Xt, ot, a, node_cols(gnodes[a]), ok, 1e-6, 256, 1024, 0)
                           for a in picks])
    for a, o in zip(picks, onodes):
        g = gnodes[a]
        assert len(g["rows"]) == min(1024, ot.N - (int(ot.end[a]) - int(ot.begin[a])))
        kerr = gram_kerr_gaussian(Xt[g["rows"]], Xt[node_cols(g)], ot.centroid[a], 1.0)
        check_node_reduced(g, o, Xt, ok, kerr)


@pytest.mark.parametrize("xi,fmm", [(2.0, False), (1.0, True)])
def test_separated_laplace_every_node(ffc, xi, fmm):
    """The separated3 (treecode, xi = 2) and fmm3 (FMM-style, xi = 1) workloads: N=65536, d=3 N(0,I), Laplace
    1/r, leaf 256, s=256, rank cap 128, tol 1e-6, FP64: all 510 nodes, then the far field and the whole sum at
    512 sampled targets against the oracle's evaluation of the GPU's skeletons."""
    X = W.normal(65536, 3, seed=0)
    q = W.charges(65536, seed=1)
    gk, ok = gkernel(LAPLACE), okernel(LAPLACE)
    t = ffc.build_tree(X, 256)
    sk = ffc.skeletonize(t, gk, tol=1e-6, max_rank=128, num_samples=256, seed=0, separation=xi)
    u, uf = (ffc.evaluate_fmm if fmm else ffc.evaluate_sum)(t, sk, gk, q)
    u, uf = u.cpu().numpy(), uf.cpu().numpy()
    ot = o_build_tree(X, 256)
    np.testing.assert_array_equal(t.arrays()["perm"], ot.perm)
    Xt = X[ot.perm]
    kinds = {"exact": 0, "valid": 0}
    gnodes = {a: sk.node(a) for a in range(1, ot.num_nodes)}
    onodes = oracle_nodes([lambda a=a: skeletonize_node(Xt, ot, a, node_cols(gnodes[a]), ok, 1e-6, 128, 256, 0,
                                                        rows=separated_rows(Xt, ot, a, 256, 0, xi))
                           for a in gnodes])
    for (a, g), o in zip(gnodes.items(), onodes):
        kinds[check_node_fp64(g, o, Xt, ok, 1e-6, 128)] += 1
    print(f"xi={xi} fmm={fmm}: nodes {kinds}")
    assert kinds["exact"] >= (1 << ot.depth)
    tg = W.subset(65536, 512, seed=2)
    ou, ouf = (fmm_evaluate if fmm else treecode_evaluate)(X, ot, gpu_skeletons(sk, ot.num_nodes), ok, q, xi,
                                                          targets=tg)
    assert rel(uf[tg], ouf) < FP64_REL
    assert rel(u[tg], ou) < FP64_REL
