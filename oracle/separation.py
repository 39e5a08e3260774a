"""Separated far fields and treecode evaluation (test infrastructure: a plain
FP64 CPU statement of what the GPU path computes; never imported by it).

Section 2 asks that sources and targets be well separated (eq. e:separated,
with a kernel-dependent tolerance delta, zero for the Gaussian) and describes
the treecode that follows: outgoing representations built upward, then, per
target, a traversal from the root that applies a node's representation when
the target is far enough from it and otherwise recurses, down to direct sums at
the leaves. Section 4.1 measures separation relative to the source ball: the
targets of a source set with centre x_c and radius rho are {y : |y - x_c| >=
xi rho}. For the Laplace kernel, whose singularity needs some separation,
Section 4.3 takes xi = 2 and 4.

Readings (the paper fixes no treecode details):

* Node ball: c_a = mean of node a's points, rho_a = their largest distance
  from c_a (the tree's centroid and radius). A point y outside node a is
  separated from a when |y - c_a|^2 >= (xi rho_a)^2, compared in squares.
  xi = 0 separates every outside point, which is the plain method.
* Rows: the s sampled rows of node a are drawn uniformly without replacement
  from the separated far set F_a (tree positions, ascending) by Floyd's
  algorithm on {0, ..., |F_a| - 1} with the node's stream; draw t is the t-th
  element of F_a. An empty F_a falls back to the plain rows (all points outside
  a), so that the node still carries its sources into its parent's columns.
* Evaluation: every target starts at both children of the root. At a node a
  that does not contain it, a target separated from a takes a's skeleton sum
  (far field) and stops there; otherwise it goes on to a's children, or, at a
  leaf, sums a's points directly (near field). A node containing the target is
  never applied: the target goes on to its children and finally sums its own
  leaf directly. With xi = 0 this is exactly the sibling cover.
"""
from __future__ import annotations

import numpy as np

from .kernels import Kernel, kernel_matrix
from .sampling import floyd_sample, sample_far_rows
from .skeleton import Skeletons, effective_samples, skeletonize_node
from .evaluate import upward_charges
from .tree import Tree


def separated_mask(Xt: np.ndarray, tree: Tree, a: int, xi: float, pos: np.ndarray | None = None) -> np.ndarray:
    """For tree positions pos (default all): outside node a and |y - c_a|^2 >= (xi rho_a)^2."""
    pos = np.arange(tree.N) if pos is None else np.asarray(pos, dtype=np.int64)
    b, e = int(tree.begin[a]), int(tree.end[a])
    outside = (pos < b) | (pos >= e)
    diff = Xt[pos] - tree.centroid[a]
    d2 = np.einsum("ij,ij->i", diff, diff)
    thr = xi * tree.radius[a]
    with np.errstate(over="ignore"):        # an infinite threshold separates nothing
        return outside & (d2 >= thr * thr)


def separated_far_set(Xt: np.ndarray, tree: Tree, a: int, xi: float) -> np.ndarray:
    """F_a: tree positions separated from node a, ascending."""
    return np.flatnonzero(separated_mask(Xt, tree, a, xi)).astype(np.int64)


def separated_rows(Xt: np.ndarray, tree: Tree, a: int, s: int, seed: int, xi: float) -> np.ndarray:
    """Uniform rows from F_a (the plain far set when F_a is empty), ascending."""
    F = separated_far_set(Xt, tree, a, xi)
    if len(F) == 0:
        return sample_far_rows(int(tree.begin[a]), int(tree.end[a]), tree.N, s, seed, a)
    return F[np.array(floyd_sample(len(F), s, seed, a), dtype=np.int64)]


def skeletonize_separated(X: np.ndarray, tree: Tree, k: Kernel, tol: float, max_rank: int, num_samples: int,
                          seed: int, xi: float) -> Skeletons:
    """skeleton.skeletonize with rows from the separated far sets."""
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    s = effective_samples(num_samples, max_rank)
    out = Skeletons()
    for level in range(tree.depth, 0, -1):
        for a in tree.level_nodes(level):
            if level == tree.depth:
                cols = np.arange(tree.begin[a], tree.end[a], dtype=np.int64)
            else:
                cols = np.concatenate([out.nodes[2 * a + 1].skel, out.nodes[2 * a + 2].skel])
            rows = separated_rows(Xt, tree, a, s, seed, xi)
            out.nodes[a] = skeletonize_node(Xt, tree, a, cols, k, tol, max_rank, s, seed, rows=rows)
    return out


def interaction_lists(Xt: np.ndarray, tree: Tree, xi: float):
    """The traversal's outcome: (far, near) with far[a] = target positions that
    apply node a's skeleton and near[a] = target positions that sum leaf a
    directly (both ascending)."""
    arrive = {1: np.arange(tree.N), 2: np.arange(tree.N)}
    far, near = {}, {}
    for level in range(1, tree.depth + 1):
        for a in tree.level_nodes(level):
            A = arrive.pop(a)
            sep = separated_mask(Xt, tree, a, xi, A) if len(A) else np.zeros(0, dtype=bool)
            far[a] = A[sep]
            rest = A[~sep]          # inside a, or outside but not separated
            if level == tree.depth:
                near[a] = rest
            else:
                arrive[2 * a + 1] = rest
                arrive[2 * a + 2] = rest
    return far, near


def treecode_evaluate(X: np.ndarray, tree: Tree, sk: Skeletons, k: Kernel, q: np.ndarray, xi: float,
                      targets: np.ndarray | None = None):
    """Return (u, u_far) in caller order; with targets (caller indices), only
    those entries, in that order (the sums of the other targets are skipped)."""
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    q_tree = np.asarray(q, dtype=np.float64)[tree.perm]
    qt = upward_charges(tree, sk, q_tree)
    far, near = interaction_lists(Xt, tree, xi)
    if targets is not None:
        keep = np.zeros(tree.N, dtype=bool)
        keep[np.argsort(tree.perm)[np.asarray(targets)]] = True
        far = {a: T[keep[T]] for a, T in far.items()}
        near = {a: T[keep[T]] for a, T in near.items()}
    u_far = np.zeros(tree.N)
    u_near = np.zeros(tree.N)
    for a in range(1, tree.num_nodes):
        T = far[a]
        J = sk.nodes[a].skel
        if len(T) and len(J):
            u_far[T] += kernel_matrix(Xt[T], Xt[J], k) @ qt[a]
    for a in tree.level_nodes(tree.depth):
        T = near[a]
        b, e = int(tree.begin[a]), int(tree.end[a])
        if len(T) and e > b:
            u_near[T] += kernel_matrix(Xt[T], Xt[b:e], k) @ q_tree[b:e]
    u = np.empty(tree.N)
    uf = np.empty(tree.N)
    u[tree.perm] = u_far + u_near
    uf[tree.perm] = u_far
    if targets is not None:
        return u[targets], uf[targets]
    return u, uf
