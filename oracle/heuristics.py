"""The paper's cheap geometric row samplers, on the learned proposal's candidate pool.

Section 3.2 proposes two heuristics in place of leverage sampling, whose exact
probabilities cost O(mn) (Section 3, "Importance sampling"), and Section 4.1.3
compares them with uniform and leverage sampling:

* distance sampling: rows drawn without replacement with probability depending
  on the target's distance to the source set;
* nearest neighbours: the targets closest to the source points, chosen
  deterministically.

Both need distances from every far target to the node, which the paper says
must themselves be approximated (trees, hashing). Here they reuse the learned
proposal's pool and geometry (`proposal.candidate_pool`,
`proposal.column_geometry`, `proposal.features`):

* distance: weights w_i = 1 / max(f0_i, 1e-12) with f0 = |y - c| / rho (c the
  centroid of the node's columns). Section 4.1.3 says "proportional to" the
  distance, Section 3.2 "inversely proportional"; the motivation (closer
  targets carry the larger rows) decides for the inverse. Without replacement
  by Efraimidis-Spirakis keys -ln(U_i) / w_i, U_i from the selection stream
  (the same generator as the learned selection), the s smallest keys;
* nearest: the s pool points with the smallest f2 = distance to the nearest
  point of the node's 256-point column subsample / rho (the nearest source
  point itself when the node has at most 256 columns), ties to the smaller
  pool position.

Nodes whose held-out error estimate exceeds fallback_tol are redone with
uniform rows, as for the learned sampler.
"""
from __future__ import annotations

import math

import numpy as np

from .cpqr_id import interpolative_decomposition
from .kernels import Kernel, kernel_matrix
from .proposal import (POOL_FACTOR, STREAM_KEYS, candidate_pool, column_geometry, features, heldout_error,
                       heldout_rows, unit_uniform)

DISTANCE, NEAREST = "distance", "nearest"


def select_rows_distance(f0: np.ndarray, pool: np.ndarray, s: int, seed: int, node: int) -> np.ndarray:
    """s pool entries without replacement, weights inversely proportional to f0; ascending."""
    P = len(pool)
    if s >= P:
        return np.sort(pool)
    keys = np.array([-math.log(unit_uniform(seed, node | STREAM_KEYS, i)) * max(float(f0[i]), 1e-12)
                     for i in range(P)])
    order = np.lexsort((np.arange(P), keys))
    return np.sort(pool[order[:s]])


def select_rows_nearest(f2: np.ndarray, pool: np.ndarray, s: int) -> np.ndarray:
    """The s pool entries with the smallest f2 (ties to the smaller position); ascending."""
    P = len(pool)
    if s >= P:
        return np.sort(pool)
    order = np.lexsort((np.arange(P), np.asarray(f2, dtype=np.float64)))
    return np.sort(pool[order[:s]])


def heuristic_rows(Xt: np.ndarray, tree, a: int, cols: np.ndarray, s: int, seed: int, kind: str,
                   pool_factor: int = POOL_FACTOR):
    """(rows, pool, f) for node a: the candidate pool, its features and the chosen rows."""
    b, e = int(tree.begin[a]), int(tree.end[a])
    pool = candidate_pool(b, e, tree.N, s, seed, a, pool_factor)
    F = features(Xt[pool], column_geometry(Xt[cols], seed, a))
    if kind == DISTANCE:
        return select_rows_distance(F[:, 0], pool, s, seed, a), pool, F
    if kind == NEAREST:
        return select_rows_nearest(F[:, 2], pool, s), pool, F
    raise ValueError(kind)


def skeletonize_heuristic(X, tree, k: Kernel, tol: float, max_rank: int, num_samples: int, seed: int, kind: str,
                          fallback_tol: float = 0.0, pool_factor: int = POOL_FACTOR):
    """Like skeleton.skeletonize with rows from a heuristic sampler. Returns (Skeletons, fallback flags)."""
    from .skeleton import NodeSkeleton, Skeletons, effective_samples, skeletonize_node
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    s = effective_samples(num_samples, max_rank)
    out = Skeletons()
    fell = {}
    for level in range(tree.depth, 0, -1):
        for a in tree.level_nodes(level):
            b, e = int(tree.begin[a]), int(tree.end[a])
            if level == tree.depth:
                cols = np.arange(b, e, dtype=np.int64)
            else:
                cols = np.concatenate([out.nodes[2 * a + 1].skel, out.nodes[2 * a + 2].skel])
            node = None
            fell[a] = False
            if len(cols) > 0:
                rows, _, _ = heuristic_rows(Xt, tree, a, cols, s, seed, kind, pool_factor)
                idd = interpolative_decomposition(kernel_matrix(Xt[rows], Xt[cols], k), tol, max_rank)
                node = NodeSkeleton(cols=cols, rows=rows, rank=idd.rank, piv=idd.piv, skel=cols[idd.skel],
                                    P=idd.P, rho=idd.rho, gap=idd.gap)
                if fallback_tol > 0:
                    Kh = kernel_matrix(Xt[heldout_rows(b, e, tree.N, seed, a)], Xt[cols], k)
                    if heldout_error(Kh, idd.skel, idd.P) > fallback_tol:
                        node = None
                        fell[a] = True
            if node is None:
                node = skeletonize_node(Xt, tree, a, cols, k, tol, max_rank, s, seed)
            out.nodes[a] = node
    return out, fell
