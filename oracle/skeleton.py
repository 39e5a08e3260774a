"""Sampled-row skeletonization of every tree node (Section 2.2, "Our approach").

For a node alpha with sources S (its columns) the method picks s of the real
targets outside alpha, forms the s x n sampled block K' = K(T_s, S) and takes
its ID (Section 2.2; Figure fig_algebraic_sampling (b)). The skeleton J and P
give the outgoing representation (Section 2.1.3, eq. e:id).

Nesting (the paper asks for child representations to be combined into the
parent's, Section 2, without fixing the scheme): a leaf's columns are its own
points; an internal node's columns are the skeleton of its left child followed
by the skeleton of its right child, each in pivot order. Nodes are processed
from the deepest level up to level 1 (the root has no far field).

Target set: all points outside alpha (separation xi = 0, Section 4.1 allows a
separated ball; the sibling cover used in evaluation needs the complement).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .cpqr_id import interpolative_decomposition
from .kernels import Kernel, kernel_matrix
from .sampling import sample_far_rows
from .tree import Tree


@dataclass
class NodeSkeleton:
    cols: np.ndarray      # tree positions of the node's columns
    rows: np.ndarray      # tree positions of the sampled targets
    rank: int
    piv: np.ndarray
    skel: np.ndarray      # tree positions of the skeleton points (pivot order)
    P: np.ndarray         # rank x len(cols)
    rho: np.ndarray
    gap: np.ndarray


@dataclass
class Skeletons:
    nodes: dict = field(default_factory=dict)   # node id -> NodeSkeleton


def effective_samples(num_samples: int, max_rank: int) -> int:
    """Default sample count: twice the rank cap when none is given."""
    return num_samples if num_samples > 0 else 2 * max_rank


def skeletonize_node(Xt: np.ndarray, tree: Tree, a: int, cols: np.ndarray, k: Kernel,
                     tol: float, max_rank: int, s: int, seed: int,
                     rows: np.ndarray | None = None) -> NodeSkeleton:
    b, e = int(tree.begin[a]), int(tree.end[a])
    if rows is None:
        rows = sample_far_rows(b, e, tree.N, s, seed, a)
    Kp = kernel_matrix(Xt[rows], Xt[cols], k)
    if len(cols) == 0 or len(rows) == 0:
        return NodeSkeleton(cols=cols, rows=rows, rank=0, piv=np.arange(len(cols)),
                            skel=cols[:0], P=np.zeros((0, len(cols))), rho=np.zeros(0),
                            gap=np.ones(0))
    idd = interpolative_decomposition(Kp, tol, max_rank)
    return NodeSkeleton(cols=cols, rows=rows, rank=idd.rank, piv=idd.piv,
                        skel=cols[idd.skel], P=idd.P, rho=idd.rho, gap=idd.gap)


def skeletonize(X: np.ndarray, tree: Tree, k: Kernel, tol: float, max_rank: int,
                num_samples: int = 0, seed: int = 0) -> Skeletons:
    """Skeletons of all non-root nodes, deepest level first."""
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    s = effective_samples(num_samples, max_rank)
    out = Skeletons()
    for level in range(tree.depth, 0, -1):
        for a in tree.level_nodes(level):
            if level == tree.depth:
                cols = np.arange(tree.begin[a], tree.end[a], dtype=np.int64)
            else:
                cols = np.concatenate([out.nodes[2 * a + 1].skel, out.nodes[2 * a + 2].skel])
            out.nodes[a] = skeletonize_node(Xt, tree, a, cols, k, tol, max_rank, s, seed)
    return out
