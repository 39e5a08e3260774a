"""The allocation-free ID entry point (ffc_interp_decomp_noalloc) through the
C ABI: two calls in a row, the second on smaller blocks, each against the
allocating ffc_interp_decomp on the same input (same bits) and against the
oracle; with every library allocation forced to fail it still runs."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.cpqr_id import interpolative_decomposition
from tests._parity import GAP_MIN

pytestmark = pytest.mark.gpu


def decaying(s, n, seed, decay=8.0):
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((s, min(s, n))))
    V, _ = np.linalg.qr(g.standard_normal((n, min(s, n))))
    return U @ np.diag(10.0 ** -np.linspace(0, decay, min(s, n))) @ V.T


def run(lib, fn, mats, tol, max_rank, stream):
    b, s, n = mats.shape
    work = torch.as_tensor(mats, device="cuda").transpose(1, 2).contiguous()   # column-major blocks
    rank = torch.full((b,), -1, dtype=torch.int32, device="cuda")
    piv = torch.full((b, n), -1, dtype=torch.int32, device="cuda")
    P = torch.zeros((b, max_rank, n), dtype=torch.float64, device="cuda")
    stream.synchronize()
    code = getattr(lib, fn)(ctypes.c_void_p(work.data_ptr()), b, s, n, tol, max_rank,
                            ctypes.c_void_p(rank.data_ptr()), ctypes.c_void_p(piv.data_ptr()),
                            ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    assert code == 0, lib.ffc_last_error()
    stream.synchronize()
    return rank.cpu().numpy(), piv.cpu().numpy(), P.cpu().numpy()


def test_noalloc_id_matches_the_allocating_call(monkeypatch):
    from paper_1409_2802_amd import ffc
    assert torch.cuda.is_available()
    lib = ffc.load_library()
    stream = torch.cuda.Stream()
    # The second call on smaller blocks; a third with more than 512 rows (32-lane groups).
    cases = [(5, 300, 200, 1e-7, 96), (3, 120, 72, 1e-6, 40), (2, 900, 160, 1e-7, 80)]
    for i, (b, s, n, tol, mr) in enumerate(cases):
        mats = np.stack([decaying(s, n, 10 * i + j) for j in range(b)])
        ref = run(lib, "ffc_interp_decomp", mats, tol, mr, stream)
        monkeypatch.setenv("FFC_FAIL_ALLOC", "1")      # any library allocation would now fail
        got = run(lib, "ffc_interp_decomp_noalloc", mats, tol, mr, stream)
        monkeypatch.delenv("FFC_FAIL_ALLOC")
        for x, y in zip(ref, got):
            np.testing.assert_array_equal(x, y)
        rank, piv, P = got
        for j in range(b):
            o = interpolative_decomposition(mats[j], tol, mr)
            assert o.gap.min() > GAP_MIN
            assert rank[j] == o.rank
            np.testing.assert_array_equal(piv[j, :rank[j]], o.piv[:o.rank])
            kappa = np.linalg.cond(o.R[:, :o.rank])
            np.testing.assert_allclose(P[j, :rank[j]], o.P, atol=max(1e-13, 1e-15 * kappa) * max(1.0, np.abs(o.P).max()))
    ffc.check_device()


def test_noalloc_id_refuses_what_it_cannot_hold():
    from paper_1409_2802_amd import ffc
    lib = ffc.load_library()
    A = torch.zeros((1100, 8), dtype=torch.float64, device="cuda")
    r = torch.zeros(1, dtype=torch.int32, device="cuda")
    pv = torch.zeros(8, dtype=torch.int32, device="cuda")
    P = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (A, r, pv, P)]
    assert lib.ffc_interp_decomp_noalloc(ptrs[0], 1, 1100, 8, 1e-6, 8, ptrs[1], ptrs[2], ptrs[3], None) == \
        ffc.FFC_ERR_INVALID_ARG
    assert b"1024" in lib.ffc_last_error()
    # More 512 x 512 blocks than the fixed scratch holds.
    assert lib.ffc_interp_decomp_noalloc(ptrs[0], 4000, 512, 512, 1e-6, 256, ptrs[1], ptrs[2], ptrs[3], None) == \
        ffc.FFC_ERR_INVALID_ARG
