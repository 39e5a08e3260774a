"""Python binding of libffc.so (argument marshalling only).

Every call goes straight to the C ABI declared in include/ffc.h; all
computation happens in the library's HIP kernels. torch tensors supply device
memory and the current HIP stream. There is no fallback: if the library is
missing or the GPU is absent, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffc.so")

FFC_OK, FFC_ERR_INVALID_ARG, FFC_ERR_HIP, FFC_ERR_OOM, FFC_ERR_NONFINITE, FFC_ERR_STATE = range(6)
GAUSSIAN, LAPLACE, POLYNOMIAL = 0, 1, 2
FP64, FP32, MIXED_BF16X3 = 0, 1, 2
SAMPLE_UNIFORM, SAMPLE_LEARNED, SAMPLE_DISTANCE, SAMPLE_NEAREST = 0, 1, 2, 3
LABEL_PIVOTED, LABEL_RIDGE = 0, 1

# Every exported entry point of include/ffc.h.
EXPORTS = [
    "ffc_build_tree", "ffc_build_partition", "ffc_tree_info", "ffc_tree_arrays",
    "ffc_skeletonize_nodes", "ffc_evaluate_sum", "ffc_evaluate_fmm", "ffc_direct_sum", "ffc_sampled_block",
    "ffc_interp_decomp", "ffc_skel_node", "ffc_skel_stats", "ffc_check_device",
    "ffc_free_tree", "ffc_free_skel", "ffc_last_error", "ffc_profile_enable", "ffc_profile_read",
    "ffc_proposal_create", "ffc_proposal_get", "ffc_proposal_free", "ffc_proposal_features",
    "ffc_proposal_fit_standardization", "ffc_proposal_score", "ffc_proposal_gradient", "ffc_proposal_adam",
    "ffc_leverage_labels", "ffc_proposal_train", "ffc_proposal_training_set",
    "ffc_step_graph_create", "ffc_step_graph_create_fmm", "ffc_graph_launch", "ffc_graph_free", "ffc_autotune_report",
    "ffc_autotune_reset",
    "ffc_skel_load", "ffc_proposal_get_adam", "ffc_proposal_set_adam", "ffc_shutdown",
    "ffc_proposal_save", "ffc_proposal_load", "ffc_pivoted_leverage_labels", "ffc_interp_decomp_noalloc",
]

NPARAM = 5313
NFEAT = 16

STAGES = ["tree", "sample", "columns", "kblock", "cpqr", "skel", "upward", "evaluate", "direct", "solve",
          "proposal", "heldout", "labels", "train"]


class FfcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ffc error {code}: {msg}")
        self.code = code


class KernelC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_int32), ("h", ctypes.c_double), ("c", ctypes.c_double)]


class SkelOptsC(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_rank", ctypes.c_int32), ("num_samples", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("sampler", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("proposal", ctypes.c_void_p), ("fallback_tol", ctypes.c_double), ("pool_factor", ctypes.c_int32),
                ("adaptive_tol", ctypes.c_double), ("max_samples", ctypes.c_int32), ("separation", ctypes.c_double)]


class StatsC(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int32), ("rank_min", ctypes.c_int32), ("rank_max", ctypes.c_int32),
                ("rank_mean", ctypes.c_double), ("rank_cap_hits", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("kernel_evals", ctypes.c_double), ("resampled", ctypes.c_int32), ("rows_max", ctypes.c_int32)]


class TrainOptsC(ctypes.Structure):
    _fields_ = [("num_blocks", ctypes.c_int32), ("block_cols", ctypes.c_int32), ("block_rows", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("eps", ctypes.c_double), ("seed", ctypes.c_uint64), ("label", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libffc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python -m paper_1409_2802_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "ffc_build_tree": [P, I64, I32, I32, P, PP],
        "ffc_build_partition": [P, I64, I32, I64, P, PP],
        "ffc_tree_info": [P, P, P, P, P],
        "ffc_tree_arrays": [P, P, P, P, P, P],
        "ffc_skeletonize_nodes": [P, ctypes.POINTER(KernelC), ctypes.POINTER(SkelOptsC), P, I32, P, PP],
        "ffc_evaluate_sum": [P, P, ctypes.POINTER(KernelC), P, P, P, I32, P],
        "ffc_evaluate_fmm": [P, P, ctypes.POINTER(KernelC), P, P, P, I32, P],
        "ffc_direct_sum": [P, I64, P, I64, I32, ctypes.POINTER(KernelC), P, P, I32, P],
        "ffc_sampled_block": [P, ctypes.POINTER(KernelC), I32, P, I32, P, I32, P, P],
        "ffc_interp_decomp": [P, I32, I32, I32, D, I32, P, P, P, P],
        "ffc_interp_decomp_noalloc": [P, I32, I32, I32, D, I32, P, P, P, P],
        "ffc_skel_node": [P, I32, P, P, P, P, P, P, P],
        "ffc_skel_stats": [P, ctypes.POINTER(StatsC)],
        "ffc_skel_load": [P, ctypes.POINTER(SkelOptsC), P, P, P, P, I32, I32, P, PP],
        "ffc_proposal_get_adam": [P, P, P, P],
        "ffc_proposal_set_adam": [P, P, P, I32],
        "ffc_check_device": [P],
        "ffc_profile_enable": [I32],
        "ffc_profile_read": [P, P, I32, I32],
        "ffc_proposal_create": [P, P, P, PP],
        "ffc_proposal_get": [P, P, P, P],
        "ffc_proposal_features": [P, P, I32, P, P, P, I32, P, I32, U64, P, P],
        "ffc_proposal_fit_standardization": [P, P, I64, P],
        "ffc_proposal_score": [P, P, I64, P, P],
        "ffc_proposal_gradient": [P, P, P, I64, P, P, P],
        "ffc_proposal_adam": [P, P, ctypes.c_float, P],
        "ffc_leverage_labels": [P, I64, I32, I32, D, P, P, P],
        "ffc_pivoted_leverage_labels": [P, I64, I32, I32, D, P, P, P, P, P],
        "ffc_proposal_train": [P, P, ctypes.POINTER(KernelC), ctypes.POINTER(TrainOptsC), P, P],
        "ffc_proposal_training_set": [P, ctypes.POINTER(KernelC), ctypes.POINTER(TrainOptsC), P, P, P, P, P, P, P,
                                      P, P],
        "ffc_step_graph_create": [P, P, ctypes.POINTER(KernelC), ctypes.POINTER(SkelOptsC), P, P, P, I32, P, PP],
        "ffc_step_graph_create_fmm": [P, P, ctypes.POINTER(KernelC), ctypes.POINTER(SkelOptsC), P, P, P, I32, P, PP],
        "ffc_graph_launch": [P, P],
        "ffc_autotune_report": [P, I32, P],
        "ffc_proposal_save": [P, ctypes.c_char_p],
        "ffc_proposal_load": [ctypes.c_char_p, PP],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ffc_free_tree.argtypes = [P]
    lib.ffc_free_tree.restype = None
    lib.ffc_free_skel.argtypes = [P]
    lib.ffc_free_skel.restype = None
    lib.ffc_graph_free.argtypes = [P]
    lib.ffc_graph_free.restype = None
    lib.ffc_proposal_free.argtypes = [P]
    lib.ffc_proposal_free.restype = None
    lib.ffc_last_error.argtypes = []
    lib.ffc_last_error.restype = ctypes.c_char_p
    lib.ffc_shutdown.argtypes = []
    lib.ffc_shutdown.restype = None
    lib.ffc_autotune_reset.argtypes = []
    lib.ffc_autotune_reset.restype = None
    _lib = lib
    return lib


# Live handles, released in a fixed order (graphs, skeleton sets, proposals,
# trees) at interpreter exit, before the library's process-wide resources are
# freed by ffc_shutdown: nothing of the library's is left for finalizers that
# run during teardown.
_live: "weakref.WeakSet" = weakref.WeakSet()
_RELEASE_ORDER = ("StepGraph", "Skeletons", "Proposal", "Tree")


def _register(obj) -> None:
    _live.add(obj)


@atexit.register
def _shutdown() -> None:
    if _lib is None:
        return
    objs = list(_live)
    for kind in _RELEASE_ORDER:
        for o in objs:
            if type(o).__name__ == kind:
                o._release()
    _lib.ffc_shutdown()


def _check(code: int) -> None:
    if code != FFC_OK:
        raise FfcError(code, load_library().ffc_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dev_f64(x, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64))
    if not x.is_cuda:
        x = x.to("cuda")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return x.contiguous()


def _dev_i32(x) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32))
    return x.to(device="cuda", dtype=torch.int32).contiguous()


@dataclass(frozen=True)
class Kernel:
    kind: int
    h: float = 1.0
    c: float = 1.0
    p: int = 1

    def c_struct(self) -> KernelC:
        return KernelC(kind=self.kind, p=self.p, h=self.h, c=self.c)


class Tree:
    """Handle to a ball tree (or two-part partition) built on the GPU."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        depth, nn, N, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(load_library().ffc_tree_info(handle, ctypes.byref(depth), ctypes.byref(nn), ctypes.byref(N),
                                            ctypes.byref(d)))
        self.depth, self.num_nodes, self.N, self.d = depth.value, nn.value, N.value, d.value
        _register(self)

    @property
    def handle(self):
        return self._h

    def arrays(self) -> dict:
        perm = np.empty(self.N, dtype=np.int32)
        b = np.empty(self.num_nodes, dtype=np.int64)
        e = np.empty(self.num_nodes, dtype=np.int64)
        cen = np.empty((self.num_nodes, self.d), dtype=np.float64)
        rad = np.empty(self.num_nodes, dtype=np.float64)
        _check(load_library().ffc_tree_arrays(self._h, perm.ctypes.data, b.ctypes.data, e.ctypes.data,
                                              cen.ctypes.data, rad.ctypes.data))
        return {"perm": perm, "begin": b, "end": e, "centroid": cen, "radius": rad}

    def _release(self) -> None:
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ffc_free_tree(self._h)
        self._h = None

    def __del__(self):
        self._release()


def build_tree(X, leaf_size: int, stream=None) -> Tree:
    Xd = _dev_f64(X, "X")
    h = ctypes.c_void_p()
    _check(load_library().ffc_build_tree(_ptr(Xd), Xd.shape[0], Xd.shape[1], leaf_size, _stream(stream),
                                         ctypes.byref(h)))
    return Tree(h)


def build_partition(X, n_left: int, stream=None) -> Tree:
    Xd = _dev_f64(X, "X")
    h = ctypes.c_void_p()
    _check(load_library().ffc_build_partition(_ptr(Xd), Xd.shape[0], Xd.shape[1], n_left, _stream(stream),
                                              ctypes.byref(h)))
    return Tree(h)


class Skeletons:
    """Handle to the per-node skeletons of a tree."""

    def __init__(self, handle: ctypes.c_void_p, tree: Tree):
        self._h = handle
        self.tree = tree
        _register(self)

    @property
    def handle(self):
        return self._h

    def node(self, a: int) -> dict:
        lib = load_library()
        r, nc, nr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.ffc_skel_node(self._h, a, ctypes.byref(r), ctypes.byref(nc), ctypes.byref(nr), None, None, None,
                                 None))
        cols = np.empty(max(nc.value, 1), dtype=np.int32)
        rows = np.empty(max(nr.value, 1), dtype=np.int32)
        skel = np.empty(max(r.value, 1), dtype=np.int32)
        P = np.empty((max(r.value, 1), max(nc.value, 1)), dtype=np.float64)
        _check(lib.ffc_skel_node(self._h, a, ctypes.byref(r), ctypes.byref(nc), ctypes.byref(nr), cols.ctypes.data,
                                 rows.ctypes.data, skel.ctypes.data, P.ctypes.data))
        return {"rank": r.value, "cols": cols[:nc.value], "rows": rows[:nr.value], "skel": skel[:r.value],
                "P": P[:r.value, :nc.value]}

    def stats(self) -> dict:
        st = StatsC()
        _check(load_library().ffc_skel_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in StatsC._fields_}

    def export(self) -> dict:
        """Every node's rank, column count, skeleton and P in the padded layout of ffc_skel_load."""
        nn = self.tree.num_nodes
        nodes = {a: self.node(a) for a in range(1, nn)}
        r_max = max([1] + [v["rank"] for v in nodes.values()])
        n_max = max([1] + [len(v["cols"]) for v in nodes.values()])
        rank = np.zeros(nn, dtype=np.int32)
        ncols = np.zeros(nn, dtype=np.int32)
        skel = np.zeros((nn, r_max), dtype=np.int32)
        P = np.zeros((nn, r_max, n_max), dtype=np.float64)
        for a, v in nodes.items():
            r, n = v["rank"], len(v["cols"])
            rank[a], ncols[a] = r, n
            skel[a, :r] = v["skel"]
            P[a, :r, :n] = v["P"]
        return {"rank": rank, "ncols": ncols, "skel": skel, "P": P}

    def save(self, path: str, separation: float = 0.0) -> None:
        """Checkpoint (numpy .npz of plain arrays) that load_skeletons reads back."""
        np.savez(path, separation=np.float64(separation), **self.export())

    def _release(self) -> None:
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ffc_free_skel(self._h)
        self._h = None

    def __del__(self):
        self._release()


def load_skeletons(tree: Tree, source, separation: float | None = None, stream=None) -> Skeletons:
    """A skeleton set from Skeletons.export() arrays or a Skeletons.save() checkpoint, for evaluation."""
    if isinstance(source, (str, os.PathLike)):
        with np.load(source, allow_pickle=False) as z:
            source = {k: z[k] for k in z.files}
    if separation is None:
        separation = float(source.get("separation", 0.0))
    rank = np.ascontiguousarray(source["rank"], dtype=np.int32)
    ncols = np.ascontiguousarray(source["ncols"], dtype=np.int32)
    skel = np.ascontiguousarray(source["skel"], dtype=np.int32)
    P = np.ascontiguousarray(source["P"], dtype=np.float64)
    if rank.shape != (tree.num_nodes,) or skel.shape[0] != tree.num_nodes or P.shape[:2] != skel.shape:
        raise ValueError("checkpoint arrays do not match the tree")
    opts = SkelOptsC(separation=separation)
    h = ctypes.c_void_p()
    _check(load_library().ffc_skel_load(tree.handle, ctypes.byref(opts), rank.ctypes.data, ncols.ctypes.data,
                                        skel.ctypes.data, P.ctypes.data, skel.shape[1], P.shape[2], _stream(stream),
                                        ctypes.byref(h)))
    return Skeletons(h, tree)


def skeletonize(tree: Tree, kernel: Kernel, tol: float, max_rank: int, num_samples: int = 0,
                precision: int = FP64, seed: int = 0, reuse: Skeletons | None = None,
                proposal: "Proposal | None" = None, fallback_tol: float = 0.0, pool_factor: int = 0,
                adaptive_tol: float = 0.0, max_samples: int = 0, sampler: int | None = None,
                separation: float = 0.0, node_ids=None, stream=None) -> Skeletons:
    """Skeletonize every non-root node; with `proposal` the rows come from the learned sampler (or `sampler`:
    SAMPLE_DISTANCE / SAMPLE_NEAREST for the paper's heuristics on the same candidate pool), with
    `adaptive_tol` > 0 a node's row count doubles until its held-out error estimate is at most adaptive_tol
    (or `max_samples` is reached); with `separation` xi > 0 the rows come from each node's separated points
    and evaluate_sum runs the treecode; `node_ids` restricts the call to those nodes (the others keep what
    `reuse` holds)."""
    if sampler is None:
        sampler = SAMPLE_LEARNED if proposal is not None else SAMPLE_UNIFORM
    opts = SkelOptsC(tol=tol, max_rank=max_rank, num_samples=num_samples, precision=precision,
                     sampler=sampler, seed=seed,
                     proposal=proposal.handle if proposal is not None else None, fallback_tol=fallback_tol,
                     pool_factor=pool_factor, adaptive_tol=adaptive_tol, max_samples=max_samples,
                     separation=separation)
    h = ctypes.c_void_p(reuse.handle.value if reuse is not None else None)
    k = kernel.c_struct()
    ids = None if node_ids is None else np.ascontiguousarray(node_ids, dtype=np.int32)
    _check(load_library().ffc_skeletonize_nodes(tree.handle, ctypes.byref(k), ctypes.byref(opts),
                                                None if ids is None else ids.ctypes.data,
                                                0 if ids is None else len(ids), _stream(stream), ctypes.byref(h)))
    if reuse is not None:
        return reuse
    return Skeletons(h, tree)


class StepGraph:
    """One step (skeletonize with reuse + evaluate) captured as a HIP graph; fmm selects the FMM-style
    evaluation (after one eager evaluate_fmm at the same separation)."""

    def __init__(self, tree: Tree, sk: Skeletons, kernel: Kernel, q: torch.Tensor, u: torch.Tensor,
                 u_far: torch.Tensor | None, stream, tol: float, max_rank: int, num_samples: int = 0,
                 precision: int = FP64, seed: int = 0, proposal: "Proposal | None" = None, pool_factor: int = 0,
                 sampler: int | None = None, separation: float = 0.0, fmm: bool = False):
        if sampler is None:
            sampler = SAMPLE_LEARNED if proposal is not None else SAMPLE_UNIFORM
        opts = SkelOptsC(tol=tol, max_rank=max_rank, num_samples=num_samples, precision=precision,
                         sampler=sampler, seed=seed,
                         proposal=proposal.handle if proposal is not None else None, fallback_tol=0.0,
                         pool_factor=pool_factor, separation=separation)
        self._keep = (tree, sk, q, u, u_far, proposal)   # the graph holds their device pointers
        k = kernel.c_struct()
        h = ctypes.c_void_p()
        create = load_library().ffc_step_graph_create_fmm if fmm else load_library().ffc_step_graph_create
        _check(create(tree.handle, sk.handle, ctypes.byref(k), ctypes.byref(opts), _ptr(q), _ptr(u), _ptr(u_far),
                      precision, _stream(stream), ctypes.byref(h)))
        self._h = h
        _register(self)

    def launch(self, stream=None) -> None:
        _check(load_library().ffc_graph_launch(self._h, _stream(stream)))

    def _release(self) -> None:
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ffc_graph_free(self._h)
        self._h = None

    def free(self) -> None:
        """Release the graph now (ffc_graph_free): while it lives, calls that would resize or replace the buffers
        it holds on its tree and skeletons are refused."""
        self._release()

    def __del__(self):
        self._release()


def evaluate_sum(tree: Tree, sk: Skeletons, kernel: Kernel, q, precision: int = FP64, stream=None):
    qd = _dev_f64(q, "q")
    u = torch.empty(tree.N, dtype=torch.float64, device="cuda")
    uf = torch.empty(tree.N, dtype=torch.float64, device="cuda")
    k = kernel.c_struct()
    _check(load_library().ffc_evaluate_sum(tree.handle, sk.handle, ctypes.byref(k), _ptr(qd), _ptr(u), _ptr(uf),
                                           precision, _stream(stream)))
    return u, uf


def evaluate_fmm(tree: Tree, sk: Skeletons, kernel: Kernel, q, precision: int = FP64, stream=None):
    """FMM-style evaluation (incoming representations from the skeletons); returns (u, u_far)."""
    qd = _dev_f64(q, "q")
    u = torch.empty(tree.N, dtype=torch.float64, device="cuda")
    uf = torch.empty(tree.N, dtype=torch.float64, device="cuda")
    evaluate_fmm_into(tree, sk, kernel, qd, u, uf, precision, stream)
    return u, uf


def evaluate_fmm_into(tree: Tree, sk: Skeletons, kernel: Kernel, q: torch.Tensor, u: torch.Tensor,
                      u_far: torch.Tensor | None, precision: int = FP64, stream=None) -> None:
    k = kernel.c_struct()
    _check(load_library().ffc_evaluate_fmm(tree.handle, sk.handle, ctypes.byref(k), _ptr(q), _ptr(u), _ptr(u_far),
                                           precision, _stream(stream)))


def evaluate_sum_into(tree: Tree, sk: Skeletons, kernel: Kernel, q: torch.Tensor, u: torch.Tensor,
                      u_far: torch.Tensor | None, precision: int = FP64, stream=None) -> None:
    k = kernel.c_struct()
    _check(load_library().ffc_evaluate_sum(tree.handle, sk.handle, ctypes.byref(k), _ptr(q), _ptr(u), _ptr(u_far),
                                           precision, _stream(stream)))


def direct_sum(Y, X, q, kernel: Kernel, precision: int = FP64, out: torch.Tensor | None = None, stream=None):
    Yd, Xd, qd = _dev_f64(Y, "Y"), _dev_f64(X, "X"), _dev_f64(q, "q")
    if Yd.shape[1] != Xd.shape[1] or qd.shape[0] != Xd.shape[0]:
        raise ValueError("shape mismatch")
    u = out if out is not None else torch.empty(Yd.shape[0], dtype=torch.float64, device="cuda")
    k = kernel.c_struct()
    _check(load_library().ffc_direct_sum(_ptr(Yd), Yd.shape[0], _ptr(Xd), Xd.shape[0], Xd.shape[1], ctypes.byref(k),
                                         _ptr(qd), _ptr(u), precision, _stream(stream)))
    return u


def sampled_block(tree: Tree, kernel: Kernel, rows, cols, precision: int = FP64, stream=None) -> torch.Tensor:
    """K(x_rows, x_cols) for tree positions; returned as an (s, n) view."""
    rd, cd = _dev_i32(rows), _dev_i32(cols)
    s, n = rd.numel(), cd.numel()
    out = torch.empty((n, s), dtype=torch.float64, device="cuda")
    k = kernel.c_struct()
    _check(load_library().ffc_sampled_block(tree.handle, ctypes.byref(k), precision, _ptr(rd), s, _ptr(cd), n,
                                            _ptr(out), _stream(stream)))
    return out.T


def interp_decomp(A, tol: float, max_rank: int, stream=None):
    """Batched ID of A (batch, s, n). Returns (rank[b], piv[b, n], P[b, max_rank, n])."""
    Ad = _dev_f64(A, "A")
    if Ad.dim() == 2:
        Ad = Ad[None]
    b, s, n = Ad.shape
    work = Ad.transpose(1, 2).contiguous()          # column-major s x n blocks
    rank = torch.zeros(b, dtype=torch.int32, device="cuda")
    piv = torch.zeros((b, n), dtype=torch.int32, device="cuda")
    P = torch.zeros((b, max_rank, n), dtype=torch.float64, device="cuda")
    _check(load_library().ffc_interp_decomp(_ptr(work), b, s, n, tol, max_rank, _ptr(rank), _ptr(piv), _ptr(P),
                                            _stream(stream)))
    return rank, piv, P


def check_device(stream=None) -> None:
    """Raise FfcError(FFC_ERR_NONFINITE) if a kernel value was not finite."""
    _check(load_library().ffc_check_device(_stream(stream)))


def profile_enable(on: bool = True) -> None:
    _check(load_library().ffc_profile_enable(1 if on else 0))


def profile_read(reset: bool = True) -> dict:
    """Accumulated milliseconds and launch counts per stage since the last reset."""
    n = len(STAGES)
    ms = np.zeros(n, dtype=np.float64)
    cnt = np.zeros(n, dtype=np.int64)
    _check(load_library().ffc_profile_read(ms.ctypes.data, cnt.ctypes.data, n, 1 if reset else 0))
    return {name: {"ms": float(ms[i]), "launches": int(cnt[i])} for i, name in enumerate(STAGES)}


# ---------------------------------------------------------------------------
# Learned row proposal
# ---------------------------------------------------------------------------
def _dev_f32(x, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32))
    if not x.is_cuda:
        x = x.to("cuda")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return x.contiguous()


class Proposal:
    """Handle to the 16-64-64-1 proposal network (parameters, standardization, Adam state)."""

    def __init__(self, theta, mu=None, sd=None, _handle=None):
        if _handle is not None:   # from ffc_proposal_load
            self._h = _handle
            _register(self)
            return
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.shape != (NPARAM,):
            raise ValueError(f"theta must have {NPARAM} entries")
        m = None if mu is None else np.ascontiguousarray(mu, dtype=np.float32)
        v = None if sd is None else np.ascontiguousarray(sd, dtype=np.float32)
        h = ctypes.c_void_p()
        _check(load_library().ffc_proposal_create(th.ctypes.data, None if m is None else m.ctypes.data,
                                                  None if v is None else v.ctypes.data, ctypes.byref(h)))
        self._h = h
        _register(self)

    @property
    def handle(self):
        return self._h

    def get(self):
        th = np.empty(NPARAM, dtype=np.float32)
        mu = np.empty(NFEAT, dtype=np.float32)
        sd = np.empty(NFEAT, dtype=np.float32)
        _check(load_library().ffc_proposal_get(self._h, th.ctypes.data, mu.ctypes.data, sd.ctypes.data))
        return th, mu, sd

    def adam_state(self):
        m1 = np.empty(NPARAM, dtype=np.float32)
        m2 = np.empty(NPARAM, dtype=np.float32)
        step = ctypes.c_int32()
        _check(load_library().ffc_proposal_get_adam(self._h, m1.ctypes.data, m2.ctypes.data, ctypes.byref(step)))
        return m1, m2, step.value

    def set_adam_state(self, m1, m2, step: int) -> None:
        a = np.ascontiguousarray(m1, dtype=np.float32)
        b = np.ascontiguousarray(m2, dtype=np.float32)
        if a.shape != (NPARAM,) or b.shape != (NPARAM,):
            raise ValueError(f"moments must have {NPARAM} entries")
        _check(load_library().ffc_proposal_set_adam(self._h, a.ctypes.data, b.ctypes.data, int(step)))

    def save(self, path: str) -> None:
        """Checkpoint of parameters, standardization and Adam state: the library's versioned binary
        (ffc_proposal_save), or a numpy .npz mirror of the same arrays when the name ends in .npz."""
        if str(path).endswith(".npz"):
            th, mu, sd = self.get()
            m1, m2, step = self.adam_state()
            np.savez(path, theta=th, mu=mu, sd=sd, m1=m1, m2=m2, step=np.int32(step))
        else:
            _check(load_library().ffc_proposal_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str) -> "Proposal":
        if str(path).endswith(".npz"):
            with np.load(path, allow_pickle=False) as z:
                p = cls(z["theta"], z["mu"], z["sd"])
                p.set_adam_state(z["m1"], z["m2"], int(z["step"]))
            return p
        h = ctypes.c_void_p()
        _check(load_library().ffc_proposal_load(os.fsencode(path), ctypes.byref(h)))
        return cls(None, _handle=h)

    def fit_standardization(self, feat: torch.Tensor, stream=None) -> None:
        f = _dev_f32(feat, "feat")
        _check(load_library().ffc_proposal_fit_standardization(self._h, _ptr(f), f.shape[0], _stream(stream)))

    def score(self, feat: torch.Tensor, stream=None) -> torch.Tensor:
        f = _dev_f32(feat, "feat")
        out = torch.empty(f.shape[0], dtype=torch.float32, device="cuda")
        _check(load_library().ffc_proposal_score(self._h, _ptr(f), f.shape[0], _ptr(out), _stream(stream)))
        return out

    def gradient(self, feat: torch.Tensor, target: torch.Tensor, stream=None):
        f, t = _dev_f32(feat, "feat"), _dev_f32(target, "target")
        g = torch.empty(NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(load_library().ffc_proposal_gradient(self._h, _ptr(f), _ptr(t), f.shape[0], _ptr(g), _ptr(loss),
                                                    _stream(stream)))
        return float(loss.item()), g

    def adam(self, grad: torch.Tensor, lr: float, stream=None) -> None:
        g = _dev_f32(grad, "grad")
        _check(load_library().ffc_proposal_adam(self._h, _ptr(g), lr, _stream(stream)))

    def train(self, tree: Tree, kernel: Kernel, num_blocks: int, block_cols: int, block_rows: int, epochs: int,
              batch: int, lr: float, eps: float, seed: int = 0, label: int = LABEL_PIVOTED,
              stream=None) -> np.ndarray:
        """Builds the training set on the GPU and trains; returns the per-epoch loss."""
        o = TrainOptsC(num_blocks=num_blocks, block_cols=block_cols, block_rows=block_rows, epochs=epochs,
                       batch=batch, lr=lr, eps=eps, seed=seed, label=label)
        loss = np.zeros(max(epochs, 1), dtype=np.float32)
        k = kernel.c_struct()
        _check(load_library().ffc_proposal_train(self._h, tree.handle, ctypes.byref(k), ctypes.byref(o),
                                                 loss.ctypes.data, _stream(stream)))
        return loss[:epochs]

    def _release(self) -> None:
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ffc_proposal_free(self._h)
        self._h = None

    def __del__(self):
        self._release()


def proposal_features(tree: Tree, cols, ncols, ids, tgt, ntgt, seed: int, stream=None) -> torch.Tensor:
    """Features (count, tgt_stride, 16) of targets tgt[g, :ntgt[g]] against columns cols[g, :ncols[g]]."""
    cd, nc, idd, td, nt = _dev_i32(cols), _dev_i32(ncols), _dev_i32(ids), _dev_i32(tgt), _dev_i32(ntgt)
    count, col_stride = cd.shape
    tgt_stride = td.shape[1]
    feat = torch.full((count, tgt_stride, NFEAT), float("nan"), dtype=torch.float32, device="cuda")
    _check(load_library().ffc_proposal_features(tree.handle, _ptr(cd), col_stride, _ptr(nc), _ptr(idd), _ptr(td),
                                                tgt_stride, _ptr(nt), count, seed, _ptr(feat), _stream(stream)))
    return feat


def leverage_labels(B, eps: float, stream=None):
    """Ridge leverages and targets of the rows of blocks B (count, m, n)."""
    Bd = _dev_f64(B, "B")
    if Bd.dim() == 2:
        Bd = Bd[None]
    count, m, n = Bd.shape
    lev = torch.empty((count, m), dtype=torch.float64, device="cuda")
    tgt = torch.empty((count, m), dtype=torch.float32, device="cuda")
    _check(load_library().ffc_leverage_labels(_ptr(Bd), m, n, count, eps, _ptr(lev), _ptr(tgt), _stream(stream)))
    return lev, tgt


def pivoted_leverage_labels(B, eps: float, stream=None):
    """Leverage at each block's eps-rank from its column-pivoted QR: (lev, targets, ranks, pivot order)."""
    Bd = _dev_f64(B, "B")
    if Bd.dim() == 2:
        Bd = Bd[None]
    count, m, n = Bd.shape
    lev = torch.empty((count, m), dtype=torch.float64, device="cuda")
    tgt = torch.empty((count, m), dtype=torch.float32, device="cuda")
    rank = np.zeros(count, dtype=np.int32)
    piv = np.zeros((count, n), dtype=np.int32)
    _check(load_library().ffc_pivoted_leverage_labels(_ptr(Bd), m, n, count, eps, _ptr(lev), _ptr(tgt),
                                                      rank.ctypes.data, piv.ctypes.data, _stream(stream)))
    return lev, tgt, rank, piv


def training_set(tree: Tree, kernel: Kernel, num_blocks: int, block_cols: int, block_rows: int, eps: float,
                 seed: int = 0, label: int = LABEL_PIVOTED, stream=None) -> dict:
    """The proposal's training set as built on the GPU (leaves, columns, targets, features, labels)."""
    o = TrainOptsC(num_blocks=num_blocks, block_cols=block_cols, block_rows=block_rows, epochs=0, batch=1, lr=1e-3,
                   eps=eps, seed=seed, label=label)
    k = kernel.c_struct()
    n, m = ctypes.c_int32(), ctypes.c_int32()
    lib = load_library()
    _check(lib.ffc_proposal_training_set(tree.handle, ctypes.byref(k), ctypes.byref(o), ctypes.byref(n),
                                         ctypes.byref(m), None, None, None, None, None, None, _stream(stream)))
    n, m = n.value, m.value
    G = num_blocks
    leaves = torch.empty(G, dtype=torch.int32, device="cuda")
    cols = torch.empty((G, n), dtype=torch.int32, device="cuda")
    rows = torch.empty((G, m), dtype=torch.int32, device="cuda")
    feat = torch.empty((G * m, NFEAT), dtype=torch.float32, device="cuda")
    tgt = torch.empty(G * m, dtype=torch.float32, device="cuda")
    lev = torch.empty(G * m, dtype=torch.float64, device="cuda")
    _check(lib.ffc_proposal_training_set(tree.handle, ctypes.byref(k), ctypes.byref(o), None, None, _ptr(leaves),
                                         _ptr(cols), _ptr(rows), _ptr(feat), _ptr(tgt), _ptr(lev), _stream(stream)))
    return {"n": n, "m": m, "leaves": leaves, "cols": cols, "rows": rows, "feat": feat, "target": tgt, "lev": lev}


def autotune_reset() -> None:
    """Forget the QR autotuner's choices in this process (FFC_TUNE_CACHE is read again on next use)."""
    load_library().ffc_autotune_reset()


def autotune_report() -> list:
    """The QR autotuner's choices so far (one dict per block shape)."""
    lib = load_library()
    cnt = ctypes.c_int32()
    _check(lib.ffc_autotune_report(None, 0, ctypes.byref(cnt)))
    buf = np.zeros(8 * max(cnt.value, 1), dtype=np.int32)
    _check(lib.ffc_autotune_report(buf.ctypes.data, cnt.value, ctypes.byref(cnt)))
    keys = ["s_max", "n_max", "batch", "max_rank", "variant", "threads", "best_us", "first_us"]
    out = []
    for e in range(cnt.value):
        rec = dict(zip(keys, map(int, buf[8 * e:8 * e + 8])))
        v = rec.pop("variant")
        rec["max_rows"], rec["cols_per_lane_group"] = v // 100, v % 100
        rec["from_cache"] = rec["first_us"] < 0
        out.append(rec)
    return out
