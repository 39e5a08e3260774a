"""The C-ABI library loads on the CPU and exports every symbol the header declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffc.h")
LIB = os.path.join(ROOT, "paper_1409_2802_amd", "libffc.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("ffc_build_tree", "ffc_skeletonize_nodes", "ffc_evaluate_sum", "ffc_direct_sum"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libffc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert missing == []


def test_binding_lists_every_declared_symbol():
    from paper_1409_2802_amd import ffc
    assert sorted(ffc.EXPORTS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libffc.so not built")
def test_argument_validation_without_gpu():
    """Invalid arguments are rejected before any device work, with a message."""
    from paper_1409_2802_amd import ffc
    lib = ffc.load_library()
    k = ffc.KernelC(kind=ffc.GAUSSIAN, p=1, h=-1.0, c=1.0)
    code = lib.ffc_direct_sum(None, 0, None, 0, 3, ctypes.byref(k), None, None, 0, None)
    assert code == ffc.FFC_ERR_INVALID_ARG
    assert b"bandwidth" in lib.ffc_last_error()
    k = ffc.KernelC(kind=ffc.LAPLACE, p=1, h=1.0, c=1.0)
    assert lib.ffc_direct_sum(None, 0, None, 0, 2, ctypes.byref(k), None, None, 0, None) == ffc.FFC_ERR_INVALID_ARG
    assert b"d >= 3" in lib.ffc_last_error()
    out = ctypes.c_void_p()
    assert lib.ffc_build_tree(None, 10, 3, 4, None, ctypes.byref(out)) == ffc.FFC_ERR_INVALID_ARG
    assert lib.ffc_interp_decomp(None, 1, 0, 4, 1e-3, 2, None, None, None, None) == ffc.FFC_ERR_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libffc.so not built")
def test_proposal_graph_and_label_validation_without_gpu():
    """The proposal, label, graph and autotuner entry points reject bad arguments before any device work."""
    from paper_1409_2802_amd import ffc
    lib = ffc.load_library()
    out = ctypes.c_void_p()
    assert lib.ffc_proposal_create(None, None, None, ctypes.byref(out)) == ffc.FFC_ERR_INVALID_ARG
    import numpy as np
    bad = np.full(ffc.NPARAM, np.nan, dtype=np.float32)
    assert lib.ffc_proposal_create(bad.ctypes.data, None, None, ctypes.byref(out)) == ffc.FFC_ERR_INVALID_ARG
    assert b"finite" in lib.ffc_last_error()
    assert lib.ffc_leverage_labels(None, 4, 3, 1, 0.0, None, None, None) == ffc.FFC_ERR_INVALID_ARG
    assert lib.ffc_leverage_labels(None, 0, 3, 1, 1e-3, None, None, None) == ffc.FFC_ERR_INVALID_ARG
    k = ffc.KernelC(kind=ffc.GAUSSIAN, p=1, h=1.0, c=1.0)
    o = ffc.SkelOptsC(tol=1e-6, max_rank=8, num_samples=0, precision=0, sampler=0, seed=0, proposal=None,
                      fallback_tol=0.0, pool_factor=0)
    assert lib.ffc_step_graph_create(None, None, ctypes.byref(k), ctypes.byref(o), None, None, None, 0, None,
                                     ctypes.byref(out)) == ffc.FFC_ERR_INVALID_ARG
    skel = ctypes.c_void_p()
    assert lib.ffc_skeletonize_nodes(None, ctypes.byref(k), ctypes.byref(o), None, 0, None, ctypes.byref(skel)) == \
        ffc.FFC_ERR_INVALID_ARG
    assert b"tree" in lib.ffc_last_error()
    assert lib.ffc_autotune_report(None, 0, None) == ffc.FFC_ERR_INVALID_ARG
    t = ffc.TrainOptsC(num_blocks=0, block_cols=8, block_rows=8, epochs=1, batch=8, lr=1e-3, eps=1e-3, seed=0)
    assert lib.ffc_proposal_train(None, None, ctypes.byref(k), ctypes.byref(t), None, None) == \
        ffc.FFC_ERR_INVALID_ARG
