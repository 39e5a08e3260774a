"""Binary ball tree grouping the points (Section 2: space-partitioning trees
define the groups whose far fields are compressed; the paper leaves the
construction open).

Reading used by the method:
* The tree is perfect: depth D is the least D >= 0 with ceil(N / 2^D) <=
  leaf_size, so every leaf sits at level D. Node ids are breadth first: the
  root is 0, the children of node a are 2a + 1 and 2a + 2.
* A node is split at the median of the projections of its points onto
  (p2 - p1), where p1 is the point farthest from the node centroid c and p2 is
  the point farthest from p1 (ties: smallest original index). The projection
  of x is (x - c) . (p2 - p1). Points are reordered ascending by (projection,
  original index); the left child takes the first ceil(n / 2) of them.
* Each node stores its range [begin, end) in tree order, its centroid (mean)
  and its radius (largest distance from the centroid).

A two-part partition (sources = one contiguous range, targets = the rest) is
the depth-1 special case with a given split and no reordering.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Tree:
    N: int
    d: int
    depth: int
    perm: np.ndarray      # perm[pos] = caller index of the point at tree position pos
    begin: np.ndarray
    end: np.ndarray
    centroid: np.ndarray  # (num_nodes, d)
    radius: np.ndarray

    @property
    def num_nodes(self) -> int:
        return len(self.begin)

    def level_nodes(self, level: int) -> range:
        return range((1 << level) - 1, (1 << (level + 1)) - 1)

    def leaf_of_position(self) -> np.ndarray:
        """Leaf node id of every tree position."""
        leaf = np.empty(self.N, dtype=np.int64)
        for a in self.level_nodes(self.depth):
            leaf[self.begin[a]:self.end[a]] = a
        return leaf


def tree_depth(N: int, leaf_size: int) -> int:
    D = 0
    while -(-N // (1 << D)) > leaf_size:
        D += 1
    return D


def _farthest(P: np.ndarray, idx: np.ndarray, ref: np.ndarray) -> int:
    d2 = ((P - ref) ** 2).sum(axis=1)
    cand = np.flatnonzero(d2 == d2.max())
    return int(cand[np.argmin(idx[cand])])


def _node_stats(X: np.ndarray, perm: np.ndarray, begin, end):
    nn = len(begin)
    d = X.shape[1]
    cen = np.zeros((nn, d))
    rad = np.zeros(nn)
    for a in range(nn):
        b, e = begin[a], end[a]
        if e > b:
            P = X[perm[b:e]]
            cen[a] = P.mean(axis=0)
            rad[a] = np.sqrt(((P - cen[a]) ** 2).sum(axis=1).max())
    return cen, rad


def build_tree(X: np.ndarray, leaf_size: int) -> Tree:
    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    D = tree_depth(N, leaf_size)
    nn = (1 << (D + 1)) - 1
    begin = np.zeros(nn, dtype=np.int64)
    end = np.zeros(nn, dtype=np.int64)
    end[0] = N
    perm = np.arange(N)
    for level in range(D):
        for a in range((1 << level) - 1, (1 << (level + 1)) - 1):
            b, e = int(begin[a]), int(end[a])
            idx = perm[b:e].copy()
            if e - b >= 2:
                P = X[idx]
                c = P.mean(axis=0)
                i1 = _farthest(P, idx, c)
                i2 = _farthest(P, idx, P[i1])
                proj = (P - c) @ (P[i2] - P[i1])
                order = np.lexsort((idx, proj))
                perm[b:e] = idx[order]
            nl = (e - b + 1) // 2
            begin[2 * a + 1], end[2 * a + 1] = b, b + nl
            begin[2 * a + 2], end[2 * a + 2] = b + nl, e
    cen, rad = _node_stats(X, perm, begin, end)
    return Tree(N=N, d=d, depth=D, perm=perm, begin=begin, end=end, centroid=cen, radius=rad)


def build_partition(X: np.ndarray, n_left: int) -> Tree:
    """Root plus two leaves: [0, n_left) and [n_left, N), caller order kept."""
    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    perm = np.arange(N)
    begin = np.array([0, 0, n_left], dtype=np.int64)
    end = np.array([N, n_left, N], dtype=np.int64)
    cen, rad = _node_stats(X, perm, begin, end)
    return Tree(N=N, d=d, depth=1, perm=perm, begin=begin, end=end, centroid=cen, radius=rad)
