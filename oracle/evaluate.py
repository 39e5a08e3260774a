"""Applying the skeletons in the kernel sum (Section 2.1.3, eq. e:id).

Equivalent charges: q~ = P q (Section 2.1.3). For an internal node the charges
of its columns are the children's equivalent charges (nesting).

Far field: the paper gives no interaction list (treecode integration is left
to other work, Section 1.2), so the reading is the sibling cover: for a target
in leaf L, the far field is the union of sibling(beta) over every beta on the
path from L up to (not including) the root. These siblings partition exactly
the points outside L, and node alpha's representation is applied to the
targets in sibling(alpha):
    u_far(y) = sum_{alpha in cover(y)} sum_j K(y, x~_{alpha,j}) q~_{alpha,j}.
Near field: the points of the target's own leaf, summed directly (Laplace:
zero-distance pairs contribute 0).
"""
from __future__ import annotations

import numpy as np

from .kernels import Kernel, kernel_matrix
from .skeleton import Skeletons
from .tree import Tree


def sibling(a: int) -> int:
    return a + 1 if a % 2 == 1 else a - 1


def upward_charges(tree: Tree, sk: Skeletons, q_tree: np.ndarray) -> dict:
    """q~_alpha = P_alpha q_alpha for every non-root node, leaves first."""
    qt = {}
    for level in range(tree.depth, 0, -1):
        for a in tree.level_nodes(level):
            if level == tree.depth:
                qa = q_tree[tree.begin[a]:tree.end[a]]
            else:
                qa = np.concatenate([qt[2 * a + 1], qt[2 * a + 2]])
            qt[a] = sk.nodes[a].P @ qa
    return qt


def evaluate(X: np.ndarray, tree: Tree, sk: Skeletons, k: Kernel, q: np.ndarray):
    """Return (u, u_far) in caller order."""
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    q_tree = np.asarray(q, dtype=np.float64)[tree.perm]
    qt = upward_charges(tree, sk, q_tree)
    u_far = np.zeros(tree.N)
    for a in range(1, tree.num_nodes):
        t = sibling(a)
        tb, te = tree.begin[t], tree.end[t]
        J = sk.nodes[a].skel
        if te > tb and len(J) > 0:
            u_far[tb:te] += kernel_matrix(Xt[tb:te], Xt[J], k) @ qt[a]
    u_near = np.zeros(tree.N)
    for a in tree.level_nodes(tree.depth):
        b, e = tree.begin[a], tree.end[a]
        if e > b:
            u_near[b:e] = kernel_matrix(Xt[b:e], Xt[b:e], k) @ q_tree[b:e]
    u = np.empty(tree.N)
    uf = np.empty(tree.N)
    u[tree.perm] = u_far + u_near
    uf[tree.perm] = u_far
    return u, uf


def exact_far_field(X: np.ndarray, tree: Tree, k: Kernel, q: np.ndarray,
                    targets: np.ndarray | None = None) -> np.ndarray:
    """Exact far field sum_{x_j outside leaf(y_i)} K(y_i, x_j) q_j (caller order).

    targets: optional caller indices; returns values for those targets only.
    """
    X = np.asarray(X, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    leaf_pos = tree.leaf_of_position()
    inv = np.empty(tree.N, dtype=np.int64)
    inv[tree.perm] = np.arange(tree.N)
    leaf_of_caller = leaf_pos[inv]
    tgt = np.arange(tree.N) if targets is None else np.asarray(targets)
    out = np.zeros(len(tgt))
    for L in np.unique(leaf_of_caller[tgt]):
        sel = np.flatnonzero(leaf_of_caller[tgt] == L)
        far = leaf_of_caller != L
        out[sel] = kernel_matrix(X[tgt[sel]], X[far], k) @ q[far]
    return out


def relative_error(approx: np.ndarray, exact: np.ndarray) -> float:
    """||approx - exact||_2 / ||exact||_2 (the paper's relative error, 2-norm)."""
    den = np.linalg.norm(exact)
    return float(np.linalg.norm(approx - exact) / den) if den > 0 else float(np.linalg.norm(approx))
