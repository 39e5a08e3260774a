"""Adaptive sample count for the sampled-row skeletonization.

The conclusion (Section 5) leaves open how many target rows to sample and
names the choice of sample count as the question of integrating the method
into a fast summation code; Section 4 fixes s as a multiple of the rank. This
module takes the direct reading of "sample until the representation is good
enough", using the same error estimate as the learned sampler's fallback:

For every node (deepest level first, columns as in `skeleton.skeletonize`):
  1. s = s0 (twice the rank cap unless given), held-out rows H = 32 uniform far
     points on their own stream (`proposal.heldout_rows`), K_h = K(H, columns);
  2. skeletonize with s uniform rows (`skeleton.skeletonize_node`, the rows a
     fresh Floyd draw of min(s, M) of the M far points);
  3. e = |K_h - K_h(:, J) P|_F / |K_h|_F (0 for an empty block);
  4. if e > adaptive_tol and the row count min(s, M) is below both the cap and
     M, set s = min(2 s, cap) and go to 2; otherwise keep this skeleton.
The cap is max_samples, or 4 s0 when that is 0.

Readings: the comparison is "e > tol means redo", as in the fallback check
(equality, a measure-zero case, counts as good enough); a larger draw is a
fresh Floyd sample, not an extension of the smaller one (Floyd's draws of
different sizes are not nested), so a node's final rows are exactly the
uniform rows of its final count.
"""
from __future__ import annotations

import numpy as np

from .kernels import Kernel, kernel_matrix
from .proposal import heldout_error, heldout_rows
from .skeleton import Skeletons, effective_samples, skeletonize_node


def adaptive_node(Xt: np.ndarray, tree, a: int, cols: np.ndarray, k: Kernel, tol: float, max_rank: int, s0: int,
                  cap: int, seed: int, adaptive_tol: float):
    """One node (Xt in tree order): returns (NodeSkeleton kept, [(rows, held-out error), ...] per draw)."""
    b, e = int(tree.begin[a]), int(tree.end[a])
    M = tree.N - (e - b)
    Kh = kernel_matrix(Xt[heldout_rows(b, e, tree.N, seed, a)], Xt[cols], k)
    s = s0
    tried = []
    while True:
        node = skeletonize_node(Xt, tree, a, cols, k, tol, max_rank, s, seed)
        err = heldout_error(Kh, node.piv[:node.rank], node.P) if len(cols) > 0 else 0.0
        nr = len(node.rows)
        tried.append((nr, err))
        if not (err > adaptive_tol and nr < cap and nr < M):
            return node, tried
        s = min(2 * s, cap)


def skeletonize_adaptive(X: np.ndarray, tree, k: Kernel, tol: float, max_rank: int, num_samples: int, seed: int,
                         adaptive_tol: float, max_samples: int = 0):
    """Skeletons of all non-root nodes with the adaptive sample count.

    Returns (Skeletons, history) with history[node] = [(rows, held-out error), ...] for every draw tried, in
    order (the last one is kept).
    """
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    s0 = effective_samples(num_samples, max_rank)
    cap = max_samples if max_samples > 0 else 4 * s0
    out = Skeletons()
    history = {}
    for level in range(tree.depth, 0, -1):
        for a in tree.level_nodes(level):
            if level == tree.depth:
                cols = np.arange(tree.begin[a], tree.end[a], dtype=np.int64)
            else:
                cols = np.concatenate([out.nodes[2 * a + 1].skel, out.nodes[2 * a + 2].skel])
            out.nodes[a], history[a] = adaptive_node(Xt, tree, a, cols, k, tol, max_rank, s0, cap, seed,
                                                     adaptive_tol)
    return out, history
