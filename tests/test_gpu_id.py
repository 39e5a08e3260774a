"""GPU batched interpolative decomposition against the oracle (Section 2.1.3,
Definition of the ID, Theorem thm_compute_id; Appendix 6.1)."""
import math

import numpy as np
import pytest
import torch

from oracle.cpqr_id import interpolative_decomposition
from oracle.kernels import POLYNOMIAL, kernel_matrix
from oracle.sampling import floyd_sample
from tests._parity import GAP_MIN, gkernel, okernel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffc():
    from paper_1409_2802_amd import ffc as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.load_library()
    return m


def decaying(s, n, seed, decay=8.0):
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((s, min(s, n))))
    V, _ = np.linalg.qr(g.standard_normal((n, min(s, n))))
    sv = 10.0 ** -np.linspace(0, decay, min(s, n))
    return U @ np.diag(sv) @ V.T


def check_against_oracle(A, rank, piv, P, tol, max_rank):
    o = interpolative_decomposition(A, tol, max_rank)
    if o.gap.size == 0 or o.gap.min() > GAP_MIN:
        assert rank == o.rank
        np.testing.assert_array_equal(piv[:rank], o.piv[:rank])
        # P agrees to the conditioning of R11 (Appendix 6.1 solve).
        R11 = o.R[:, :o.rank]
        kappa = np.linalg.cond(R11) if o.rank else 1.0
        np.testing.assert_allclose(P[:rank], o.P, atol=max(1e-13, 1e-15 * kappa) * max(1.0, np.abs(o.P).max()))
    # Reconstruction through the GPU skeleton is as good as the oracle's.
    err_g = np.linalg.norm(A - A[:, piv[:rank]] @ P[:rank])
    err_o = np.linalg.norm(A - A[:, o.skel] @ o.P)
    assert err_g <= err_o * (1 + 1e-6) + 1e-12 * np.linalg.norm(A)
    # P contains the identity on the skeleton columns.
    np.testing.assert_array_equal(P[:rank][:, piv[:rank]], np.eye(rank))


@pytest.mark.parametrize("s,n,tol,max_rank", [(40, 30, 1e-6, 30), (128, 256, 1e-6, 64), (512, 512, 1e-5, 256),
                                              (100, 7, 0.0, 7), (33, 65, 1e-3, 5), (1, 9, 1e-3, 3), (9, 1, 1e-3, 3),
                                              # 257 rows (32-row lanes), wide blocks (many workgroups per
                                              # block), and more than 512 rows (the streamed kernel)
                                              (257, 64, 1e-6, 32), (300, 1500, 1e-6, 128), (700, 300, 1e-6, 100),
                                              (1024, 50, 1e-4, 50)])
def test_batched_id_matches_oracle(ffc, s, n, tol, max_rank):
    mats = [decaying(s, n, seed) for seed in range(3)]
    rank, piv, P = ffc.interp_decomp(np.stack(mats), tol, max_rank)
    rank, piv, P = rank.cpu().numpy(), piv.cpu().numpy(), P.cpu().numpy()
    for b, A in enumerate(mats):
        check_against_oracle(A, int(rank[b]), piv[b], P[b], tol, max_rank)


def test_zero_and_full_rank_blocks(ffc):
    A = np.zeros((16, 12))
    rank, _, _ = ffc.interp_decomp(A, 1e-6, 12)
    assert int(rank[0]) == 0
    B = np.random.default_rng(0).standard_normal((20, 12))
    rank, piv, P = ffc.interp_decomp(B, 0.0, 12)
    r = int(rank[0])
    assert r == 12
    p = piv[0].cpu().numpy()
    np.testing.assert_allclose(B[:, p[:r]] @ P[0].cpu().numpy()[:r], B, atol=1e-13)


@pytest.mark.parametrize("p,expected", [(2, 15), (3, 35)])
def test_polynomial_exact_rank(ffc, p, expected):
    """(x.y/h + 1)^p in d = 4 has rank C(4 + p, p): the GPU ID finds it and the
    sampled rows reconstruct the whole block."""
    assert math.comb(4 + p, p) == expected
    g = np.random.default_rng(6)
    X, Y = g.standard_normal((80, 4)), g.standard_normal((600, 4))
    k = okernel(POLYNOMIAL, h=2.0, p=p)
    rows = np.array(floyd_sample(600, 2 * expected, seed=1, stream=0))
    rank, piv, P = ffc.interp_decomp(kernel_matrix(Y[rows], X, k), 1e-11, 80)
    r = int(rank[0])
    assert r == expected
    K = kernel_matrix(Y, X, k)
    pv = piv[0].cpu().numpy()[:r]
    assert np.linalg.norm(K - K[:, pv] @ P[0].cpu().numpy()[:r]) / np.linalg.norm(K) < 1e-9


@pytest.mark.parametrize("s,n,tol,max_rank", [(512, 512, 1e-5, 256), (256, 600, 1e-6, 128), (100, 40, 1e-8, 40),
                                              (1024, 700, 1e-6, 200), (700, 130, 1e-9, 130)])
def test_every_qr_variant_gives_the_same_bits(ffc, monkeypatch, s, n, tol, max_rank):
    """Each register-resident QR variant (lanes and rows per column, columns
    per lane group, workgroup size) that may take the blocks (16-lane groups up
    to 512 rows, 32-lane groups above), forced in turn, gives the same rank,
    pivots and P, and those match the oracle."""
    mats = np.stack([decaying(s, n, seed) for seed in (11, 12)])
    ref = None
    for v in range(11):   # every entry of the QR variant table
        monkeypatch.setenv("FFC_QR_VARIANT", str(v))
        rank, piv, P = (x.cpu().numpy() for x in ffc.interp_decomp(mats, tol, max_rank))
        if ref is None:
            ref = (rank, piv, P)
            for b, A in enumerate(mats):
                check_against_oracle(A, int(rank[b]), piv[b], P[b], tol, max_rank)
        else:
            np.testing.assert_array_equal(rank, ref[0], err_msg=f"variant {v}")
            np.testing.assert_array_equal(piv, ref[1], err_msg=f"variant {v}")
            np.testing.assert_array_equal(P, ref[2], err_msg=f"variant {v}")


@pytest.mark.parametrize("s,n", [(512, 701), (100, 90)])
def test_solve_kernels_agree_below_and_above_rank_256(ffc, s, n):
    """The interpolation solve keeps the right-hand sides in registers when the
    rank bound min(max_rank, s, n) is at most 256 and in LDS above it. With the
    rank set by the tolerance (below 256 either way) both run the same products
    in the same order: max_rank 256 and 300 give the same rank, pivots and
    bits of P, and those match the oracle."""
    decays = (14.0, 20.0, 40.0)
    mats = np.stack([decaying(s, n, seed, decay) for seed, decay in zip((21, 22, 23), decays)])
    tol = 1e-6
    outs = [tuple(x.cpu().numpy() for x in ffc.interp_decomp(mats, tol, mr)) for mr in (256, 300)]
    (r0, p0, P0), (r1, p1, P1) = outs
    assert int(r0.max()) < min(256, s, n), r0
    assert len(set(r0.tolist())) == len(decays)   # ranks of different 16-row block counts
    np.testing.assert_array_equal(r0, r1)
    np.testing.assert_array_equal(p0, p1)
    for b in range(len(mats)):   # P has max_rank rows; rows below the rank hold the solve
        r = int(r0[b])
        np.testing.assert_array_equal(P0[b, :r], P1[b, :r])
    for b, A in enumerate(mats):
        check_against_oracle(A, int(r0[b]), p0[b], P0[b], tol, 256)


def test_autotune_cache_persists_choices(ffc, tmp_path, monkeypatch):
    """With FFC_TUNE_CACHE the QR autotuner's choice is written to the file; once the process forgets its
    choices (ffc_autotune_reset, as a new process starts) it reads them back, times nothing (the report marks
    them as from the cache) and gives the same bits."""
    cache = tmp_path / "qr_tune.txt"
    monkeypatch.setenv("FFC_TUNE_CACHE", str(cache))
    monkeypatch.delenv("FFC_QR_VARIANT", raising=False)
    monkeypatch.delenv("FFC_AUTOTUNE", raising=False)
    A = np.stack([decaying(300, 200, seed) for seed in range(6)])
    outs = []
    try:
        for _ in range(2):
            ffc.autotune_reset()
            rank, piv, P = (x.cpu().numpy() for x in ffc.interp_decomp(A, 1e-7, 96))
            outs.append((rank, piv, P, ffc.autotune_report()))
    finally:
        monkeypatch.delenv("FFC_TUNE_CACHE")
        ffc.autotune_reset()
    (r0, p0, P0, rep0), (r1, p1, P1, rep1) = outs
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:5] == ["300", "200", "6", "96"]
    assert len(rep0) == 1 and not rep0[0]["from_cache"]
    assert len(rep1) == 1 and rep1[0]["from_cache"]
    for key in ("max_rows", "cols_per_lane_group", "threads"):
        assert rep0[0][key] == rep1[0][key]
    np.testing.assert_array_equal(r0, r1)
    np.testing.assert_array_equal(p0, p1)
    np.testing.assert_array_equal(P0, P1)
    for b in range(A.shape[0]):
        check_against_oracle(A[b], int(r0[b]), p0[b], P0[b], 1e-7, 96)


def test_second_process_factors_while_first_holds_cooperative_launch(ffc, tmp_path):
    """A process that has made a cooperative QR launch holds the device's cooperative-launch resource; a second
    process on the same device still factors its blocks (the one-workgroup-per-block kernel takes over when
    the cooperative launch is refused), and its results pass the oracle checks."""
    import os
    import subprocess
    import sys
    A = np.stack([decaying(300, 200, seed) for seed in range(4)])
    ffc.interp_decomp(A, 1e-7, 96)   # this process has now made cooperative launches
    torch.cuda.synchronize()
    np.save(tmp_path / "A.npy", A)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = (
        "import sys, numpy as np\n"
        f"sys.path.insert(0, {root!r})\n"
        "from paper_1409_2802_amd import ffc\n"
        f"A = np.load({str(tmp_path / 'A.npy')!r})\n"
        "r, p, P = ffc.interp_decomp(A, 1e-7, 96)\n"
        f"np.savez({str(tmp_path / 'out.npz')!r}, r=r.cpu().numpy(), p=p.cpu().numpy(), P=P.cpu().numpy())\n")
    res = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = np.load(tmp_path / "out.npz")
    for b in range(A.shape[0]):
        check_against_oracle(A[b], int(out["r"][b]), out["p"][b], out["P"][b], 1e-7, 96)
