"""FMM-style evaluation with incoming representations (test infrastructure: a
plain FP64 CPU statement of what the GPU path computes; never imported by it).

Section 2 notes that the Fast Multipole Method adds incoming representations
(the potential that distant sources induce on a group of targets) to the
treecode's outgoing ones, and that the same construction serves both. For a
symmetric kernel on one point set, the skeleton J and P of a node fitted on its
separated far field give both: outgoing K(F, cols) ~ K(F, J) P, and, by
transposition, incoming K(cols, S) ~ P^T K(J, S) for sources S in that far
field.

Readings (the paper fixes no FMM details):

* Node pairs (b, a) at one level are admissible when every point of b is
  separated from a and every point of a is separated from b (the per-point test
  of separation.py in both directions), so each side's skeleton was fitted on
  the other side's points.
* Interaction lists by the dual-tree recursion from the pairs of the root's
  children: an admissible pair of distinct nodes is a far interaction
  (multipole-to-local between skeletons); any other pair of leaves is summed
  directly; any other pair of internal nodes recurses into the four pairs of
  their children.
* Evaluation: equivalent charges q~ upward as before; v_b = sum over b's far
  list of K(x_{J_b}, x_{J_a}) q~_a at b's skeleton points; top-down, P_b^T v_b is
  added to the children's v at their skeleton points (an internal node's columns
  are its children's skeletons); at a leaf, P^T v is the far field at its
  points; the near field is the direct sum over the leaf's direct list.
"""
from __future__ import annotations

import numpy as np

from .evaluate import upward_charges
from .kernels import Kernel, kernel_matrix
from .separation import separated_mask
from .skeleton import Skeletons
from .tree import Tree


def admissible(Xt: np.ndarray, tree: Tree, b: int, a: int, xi: float) -> bool:
    """Every point of b separated from a, and every point of a from b."""
    pb = np.arange(tree.begin[b], tree.end[b])
    pa = np.arange(tree.begin[a], tree.end[a])
    return bool(separated_mask(Xt, tree, a, xi, pb).all() and separated_mask(Xt, tree, b, xi, pa).all())


def fmm_lists(Xt: np.ndarray, tree: Tree, xi: float):
    """(far, near): far[b] = source nodes of b's multipole-to-local list, near[L] = source leaves of leaf L's
    direct list, both in the order the recursion finds them (pairs by (target, source) id within a level)."""
    far = {b: [] for b in range(1, tree.num_nodes)}
    near = {L: [] for L in tree.level_nodes(tree.depth)}
    pairs = [(1, 1), (1, 2), (2, 1), (2, 2)]
    for level in range(1, tree.depth + 1):
        nxt = []
        for b, a in sorted(pairs):
            if b != a and admissible(Xt, tree, b, a, xi):
                far[b].append(a)
            elif level == tree.depth:
                near[b].append(a)
            else:
                nxt += [(cb, ca) for cb in (2 * b + 1, 2 * b + 2) for ca in (2 * a + 1, 2 * a + 2)]
        pairs = nxt
    return far, near


def fmm_evaluate(X: np.ndarray, tree: Tree, sk: Skeletons, k: Kernel, q: np.ndarray, xi: float,
                 targets: np.ndarray | None = None):
    """Return (u, u_far) in caller order; with targets (caller indices), only
    those entries, in that order (the direct leaf sums of the other targets
    are skipped)."""
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    q_tree = np.asarray(q, dtype=np.float64)[tree.perm]
    qt = upward_charges(tree, sk, q_tree)
    far, near = fmm_lists(Xt, tree, xi)
    v = {b: np.zeros(sk.nodes[b].rank) for b in range(1, tree.num_nodes)}
    for b in range(1, tree.num_nodes):
        Jb = sk.nodes[b].skel
        for a in far[b]:
            Ja = sk.nodes[a].skel
            if len(Jb) and len(Ja):
                v[b] += kernel_matrix(Xt[Jb], Xt[Ja], k) @ qt[a]
    u_far = np.zeros(tree.N)
    for level in range(1, tree.depth + 1):
        for b in tree.level_nodes(level):
            w = sk.nodes[b].P.T @ v[b]            # at b's columns
            if level == tree.depth:
                u_far[tree.begin[b]:tree.end[b]] += w
            else:
                rl = sk.nodes[2 * b + 1].rank
                v[2 * b + 1] += w[:rl]
                v[2 * b + 2] += w[rl:]
    keep = np.ones(tree.N, dtype=bool)
    if targets is not None:
        keep[:] = False
        keep[np.argsort(tree.perm)[np.asarray(targets)]] = True
    u_near = np.zeros(tree.N)
    for L, srcs in near.items():
        b, e = int(tree.begin[L]), int(tree.end[L])
        T = b + np.flatnonzero(keep[b:e])
        for a in srcs:
            ab, ae = int(tree.begin[a]), int(tree.end[a])
            if len(T):
                u_near[T] += kernel_matrix(Xt[T], Xt[ab:ae], k) @ q_tree[ab:ae]
    u = np.empty(tree.N)
    uf = np.empty(tree.N)
    u[tree.perm] = u_far + u_near
    uf[tree.perm] = u_far
    if targets is not None:
        return u[targets], uf[targets]
    return u, uf
