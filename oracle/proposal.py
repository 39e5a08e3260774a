"""Learned proposal for target-row sampling, in plain float64.

The paper samples rows uniformly, by distance, by leverage score or by nearest
neighbours (Section 4.1.3). Leverage sampling is the gold standard but needs
the whole block (Section 3, "Importance sampling"); the paper proposes cheap
geometric heuristics instead (Section 3.2). This proposal learns a map from
cheap per-target features to leverage scores and uses it for importance
sampling, with uniform sampling as a fallback.

Definitions (both sides implement these; parity unpinned for the feature set
itself, which is a design choice — its pins are invariants below):

Column set X_c (n points) of a node: centroid c = mean, radius rho = largest
distance to c (1 if zero). Subsample S: `floyd_sample(n, 256, seed, stream =
node | 2^30)` indices into the columns (all of them if n <= 256). Anchors:
a_1 = the point of S farthest from c; a_{k+1} = the point of S farthest from
{a_1..a_k} (largest minimum distance), up to 7 anchors (ties: first in S
order); u_k = (a_k - c) / |a_k - c| (0 if zero).

Features of a target y (16):
  f0 = |y - c| / rho           f1 = ln(f0 + 1e-12)
  D  = sorted |y - x| / rho over x in S
  f2..f5 = D[0..3] (D[-1] repeated if |S| < 4)
  f6 = mean D                   f7 = ln(D[0] + 1e-12)
  f8..f14 = (y - c) . u_k / rho (0 for missing anchors)
  f15 = 1

MLP 16 -> 64 (ReLU) -> 64 (ReLU) -> 1 on standardized features (f - mu) / sd
(mu, sd from the training set, sd floored at 1e-6; f15 is left as 1).
Parameters, flat: W1 (16 x 64, row-major), b1 (64), W2 (64 x 64), b2 (64),
w3 (64), b3 (1): 5313 values. Loss: mean squared error. Adam (Kingma & Ba
2015) with bias correction.

Labels (default): the leverage of Section 3 (Definition of statistical
leverage) at the block's rank, taken from the method's own column-pivoted QR
of the block B (m x n) stopped by the rank rule with tol = eps: squared row
norms of an orthonormal basis of the r pivot columns (leverage.
pivoted_leverage). Optional: the ridge leverage, lambda = eps^2 ||B||_F^2:
l_i = b_i^T (B^T B + lambda I)^{-1} b_i, i.e. sum_k U_ik^2 sigma_k^2 /
(sigma_k^2 + lambda), a smoothed form that needs no rank choice.
Target t_i = ln(max(l_i, 1e-12) * m / sum(l)).

Training set: block g (g < 2^28) picks leaf first_leaf + uniform_below(
counter(seed, 7 * 2^29, g), number of leaves); its columns are a Floyd draw
of n = min(block_cols, smallest leaf) positions inside the leaf (stream
5 * 2^29 | g), its targets a Floyd draw of m = min(block_rows, N - largest
leaf) positions outside it (stream 5 * 2^29 | 2^28 | g). Its rows' features
are taken against the geometry of its columns with stream id = the leaf, and
its labels are the targets of the ridge leverage of K(targets, columns).
Samples are numbered block-major (g m + i). Standardization: mean and
population standard deviation over all samples. Training: per epoch e, the
position p of the epoch visits sample (p * k_e) mod C (C samples), k_e = 1 +
uniform_below(counter(seed, 7 * 2^29 | 2^28, e), C - 1) raised to the next
value coprime with C; consecutive positions form mini-batches of `batch`
samples (the last one short), each followed by one Adam step.

Selection: pool of min(M, c s) uniform candidates (c = pool factor, 8 by default) (`floyd_sample` stream
node | 2^31); weights w = 0.9 softmax(score) + 0.1 / pool; Efraimidis-Spirakis
keys -ln(U_i) / w_i with U_i = ((u64 >> 11) + 0.5) 2^-53 from the counter
generator (stream node | 3 * 2^30); the s smallest keys are taken. Fallback:
32 held-out uniform rows (stream node | 2^29) estimate ||K_h - K_h(:,J) P||_F /
||K_h||_F; above fallback_tol the node is redone with uniform rows.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .cpqr_id import interpolative_decomposition
from .kernels import Kernel, kernel_matrix
from .leverage import pivoted_leverage
from .sampling import counter_u64, floyd_sample, sample_far_rows, uniform_below

NF = 16
H = 64
SUB = 256          # column subsample of the geometry
POOL_FACTOR = 8    # default candidate pool: min(M, POOL_FACTOR * s)
NPARAM = NF * H + H + H * H + H + H + 1      # 5313
STREAM_SUBSAMPLE = 1 << 30
STREAM_POOL = 1 << 31
STREAM_KEYS = 3 << 30
STREAM_HELDOUT = 1 << 29
STREAM_TRAIN_COLS = 5 << 29
STREAM_TRAIN_ROWS = (5 << 29) | (1 << 28)
STREAM_TRAIN_LEAF = 7 << 29
STREAM_TRAIN_SHUFFLE = (7 << 29) | (1 << 28)


# ----------------------------------------------------------------------------
# Features
# ----------------------------------------------------------------------------
@dataclass
class ColumnGeometry:
    c: np.ndarray
    rho: float
    S: np.ndarray          # subsample points (k x d)
    U: np.ndarray          # anchor directions (7 x d), zero rows for missing anchors


def column_geometry(Xc: np.ndarray, seed: int, node: int) -> ColumnGeometry:
    Xc = np.asarray(Xc, dtype=np.float64)
    n, d = Xc.shape
    c = Xc.mean(axis=0)
    rho = float(np.sqrt(((Xc - c) ** 2).sum(axis=1).max())) if n else 0.0
    if rho == 0.0:
        rho = 1.0
    idx = floyd_sample(n, SUB, seed, node | STREAM_SUBSAMPLE)
    S = Xc[idx]
    U = np.zeros((7, d))
    if len(S):
        chosen = []
        dist_c = ((S - c) ** 2).sum(axis=1)
        chosen.append(int(np.argmax(dist_c)))             # first maximum = first in S order
        mind = ((S - S[chosen[0]]) ** 2).sum(axis=1)
        while len(chosen) < min(7, len(S)):
            j = int(np.argmax(mind))
            chosen.append(j)
            mind = np.minimum(mind, ((S - S[j]) ** 2).sum(axis=1))
        for k, j in enumerate(chosen):
            v = S[j] - c
            nv = np.sqrt(v @ v)
            if nv > 0:
                U[k] = v / nv
    return ColumnGeometry(c=c, rho=rho, S=S, U=U)


def features(Y: np.ndarray, g: ColumnGeometry) -> np.ndarray:
    Y = np.asarray(Y, dtype=np.float64)
    m = Y.shape[0]
    F = np.zeros((m, NF))
    dc = np.sqrt(((Y - g.c) ** 2).sum(axis=1)) / g.rho
    F[:, 0] = dc
    F[:, 1] = np.log(dc + 1e-12)
    D = np.sqrt(((Y[:, None, :] - g.S[None, :, :]) ** 2).sum(axis=2)) / g.rho
    D.sort(axis=1)
    k = D.shape[1]
    for q in range(4):
        F[:, 2 + q] = D[:, min(q, k - 1)]
    F[:, 6] = D.mean(axis=1)
    F[:, 7] = np.log(D[:, 0] + 1e-12)
    F[:, 8:15] = ((Y - g.c) @ g.U.T) / g.rho
    F[:, 15] = 1.0
    return F


# ----------------------------------------------------------------------------
# MLP
# ----------------------------------------------------------------------------
def unpack(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + NF * H].reshape(NF, H); o += NF * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def standardize(F: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    Z = (np.asarray(F, dtype=np.float64) - mu) / sd
    Z[:, 15] = 1.0
    return Z


def mlp_forward(theta, Z):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    A1 = Z @ W1 + b1
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ W2 + b2
    H2 = np.maximum(A2, 0.0)
    y = H2 @ w3 + b3
    return y, (Z, A1, H1, A2, H2)


def mlp_loss_grad(theta, Z, t):
    """Mean squared error and its gradient with respect to the flat parameters."""
    y, (Z, A1, H1, A2, H2) = mlp_forward(theta, Z)
    m = len(t)
    r = y - t
    loss = float((r * r).mean())
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    dy = 2.0 * r / m
    dw3 = H2.T @ dy
    db3 = dy.sum()
    dA2 = np.outer(dy, w3) * (A2 > 0)
    dW2 = H1.T @ dA2
    db2 = dA2.sum(axis=0)
    dA1 = (dA2 @ W2.T) * (A1 > 0)
    dW1 = Z.T @ dA1
    db1 = dA1.sum(axis=0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
    return loss, grad


def adam_step(theta, m1, m2, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    mhat = m1 / (1 - b1 ** step)
    vhat = m2 / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def fit_standardization(F: np.ndarray):
    """Per-feature mean and population std (floored at 1e-6); f15 keeps mu 0, sd 1."""
    F = np.asarray(F, dtype=np.float64)
    mu = F.mean(axis=0)
    sd = np.maximum(F.std(axis=0), 1e-6)
    mu[NF - 1] = 0.0
    sd[NF - 1] = 1.0
    return mu, sd


def epoch_stride(C: int, seed: int, epoch: int) -> int:
    """Multiplier k_e of the epoch's visiting order p -> (p k_e) mod C."""
    if C <= 1:
        return 1
    k = 1 + uniform_below(counter_u64(seed, STREAM_TRAIN_SHUFFLE, epoch), C - 1)
    while math.gcd(k, C) != 1:
        k = k + 1 if k + 1 < C else 1
    return k


def train(F: np.ndarray, t: np.ndarray, theta0: np.ndarray, epochs: int, batch: int, lr: float, seed: int,
          mu: np.ndarray, sd: np.ndarray):
    """Mini-batch Adam on the mean squared error; returns (theta, per-epoch loss, per-step loss).

    The epoch loss is the sample-weighted mean of its mini-batch losses.
    """
    Z = standardize(F, mu, sd)
    t = np.asarray(t, dtype=np.float64)
    C = len(t)
    theta = np.array(theta0, dtype=np.float64)
    m1 = np.zeros_like(theta)
    m2 = np.zeros_like(theta)
    step = 0
    hist, steps = [], []
    for e in range(epochs):
        k = epoch_stride(C, seed, e)
        order = (np.arange(C, dtype=object) * k % C).astype(np.int64)
        tot = 0.0
        for p0 in range(0, C, batch):
            idx = order[p0:p0 + batch]
            loss, g = mlp_loss_grad(theta, Z[idx], t[idx])
            step += 1
            theta, m1, m2 = adam_step(theta, m1, m2, g, step, lr=lr)
            tot += loss * len(idx)
            steps.append(loss)
        hist.append(tot / C)
    return theta, np.array(hist), np.array(steps)


# ----------------------------------------------------------------------------
# Labels
# ----------------------------------------------------------------------------
def ridge_leverage(B: np.ndarray, eps: float) -> np.ndarray:
    """l_i = b_i^T (B^T B + lambda I)^{-1} b_i with lambda = eps^2 ||B||_F^2 (via the SVD)."""
    B = np.asarray(B, dtype=np.float64)
    lam = eps * eps * float((B * B).sum())
    if lam == 0.0:
        return np.zeros(B.shape[0])
    U, S, _ = np.linalg.svd(B, full_matrices=False)
    return (U * U * (S * S / (S * S + lam))).sum(axis=1)


def leverage_targets(lev: np.ndarray) -> np.ndarray:
    m = len(lev)
    tot = float(lev.sum())
    return np.log(np.maximum(lev, 1e-12) * m / max(tot, 1e-300))


# ----------------------------------------------------------------------------
# Selection
# ----------------------------------------------------------------------------
def unit_uniform(seed: int, stream: int, i: int) -> float:
    return ((counter_u64(seed, stream, i) >> 11) + 0.5) * 2.0 ** -53


def selection_keys(scores: np.ndarray, seed: int, node: int) -> np.ndarray:
    """Efraimidis-Spirakis keys -ln(U_i) / w_i of the pool entries, w = 0.9 softmax(scores) + 0.1 / pool."""
    P = len(scores)
    z = scores - scores.max()
    sm = np.exp(z) / np.exp(z).sum()
    w = 0.9 * sm + 0.1 / P
    return np.array([-math.log(unit_uniform(seed, node | STREAM_KEYS, i)) / w[i] for i in range(P)])


def select_rows(scores: np.ndarray, pool: np.ndarray, s: int, seed: int, node: int) -> np.ndarray:
    """Weighted selection without replacement of s pool entries (ES keys), ascending."""
    P = len(pool)
    if s >= P:
        return np.sort(pool)
    keys = selection_keys(scores, seed, node)
    order = np.lexsort((np.arange(P), keys))
    return np.sort(pool[order[:s]])


def candidate_pool(b: int, e: int, N: int, s: int, seed: int, node: int, factor: int = POOL_FACTOR) -> np.ndarray:
    M = N - (e - b)
    picks = floyd_sample(M, min(M, factor * s), seed, node | STREAM_POOL)
    return np.array([t if t < b else t + (e - b) for t in picks], dtype=np.int64)


def heldout_rows(b: int, e: int, N: int, seed: int, node: int) -> np.ndarray:
    M = N - (e - b)
    picks = floyd_sample(M, min(M, 32), seed, node | STREAM_HELDOUT)
    return np.array([t if t < b else t + (e - b) for t in picks], dtype=np.int64)


def heldout_error(Kh: np.ndarray, skel_local: np.ndarray, P: np.ndarray) -> float:
    den = np.linalg.norm(Kh)
    if den == 0.0:
        return 0.0
    return float(np.linalg.norm(Kh - Kh[:, skel_local] @ P) / den)


# ----------------------------------------------------------------------------
# Training set
# ----------------------------------------------------------------------------
@dataclass
class TrainingBlock:
    leaf: int
    cols: np.ndarray       # tree positions inside the leaf
    rows: np.ndarray       # tree positions outside it


def training_blocks(tree, num_blocks: int, block_cols: int, block_rows: int, seed: int):
    """The training blocks of the proposal (definitions in the module docstring)."""
    first = (1 << tree.depth) - 1
    leaves = list(tree.level_nodes(tree.depth))
    sizes = [int(tree.end[a] - tree.begin[a]) for a in leaves]
    n = min(block_cols, min(sizes))
    m = min(block_rows, tree.N - max(sizes))
    out = []
    for g in range(num_blocks):
        leaf = first + uniform_below(counter_u64(seed, STREAM_TRAIN_LEAF, g), len(leaves))
        b, e = int(tree.begin[leaf]), int(tree.end[leaf])
        cols = np.array(floyd_sample(e - b, n, seed, STREAM_TRAIN_COLS | g), dtype=np.int64) + b
        M = tree.N - (e - b)
        picks = floyd_sample(M, m, seed, STREAM_TRAIN_ROWS | g)
        rows = np.array([x if x < b else x + (e - b) for x in picks], dtype=np.int64)
        out.append(TrainingBlock(leaf=leaf, cols=cols, rows=rows))
    return out, n, m


def training_set(X, tree, k: Kernel, num_blocks: int, block_cols: int, block_rows: int, eps: float, seed: int,
                 label: str = "pivoted"):
    """Features F (C x 16), leverages and targets of all training samples, block-major. label "pivoted":
    the leverage at the block's eps-rank from its column-pivoted QR (Section 3's definition,
    leverage.pivoted_leverage); "ridge": the ridge form."""
    Xt = np.asarray(X, dtype=np.float64)[tree.perm]
    blocks, n, m = training_blocks(tree, num_blocks, block_cols, block_rows, seed)
    F, lev, tgt = [], [], []
    for blk in blocks:
        geo = column_geometry(Xt[blk.cols], seed, blk.leaf)
        F.append(features(Xt[blk.rows], geo))
        B = kernel_matrix(Xt[blk.rows], Xt[blk.cols], k)
        l = pivoted_leverage(B, eps)[0] if label == "pivoted" else ridge_leverage(B, eps)
        lev.append(l)
        tgt.append(leverage_targets(l))
    if not blocks:
        return np.zeros((0, NF)), np.zeros(0), np.zeros(0), blocks
    return np.concatenate(F), np.concatenate(lev), np.concatenate(tgt), blocks


# ----------------------------------------------------------------------------
# Learned skeletonization (Section 2.2 with importance-sampled rows)
# ----------------------------------------------------------------------------
def skeletonize_learned(X, tree, k: Kernel, tol: float, max_rank: int, num_samples: int, seed: int,
                        theta: np.ndarray, mu: np.ndarray, sd: np.ndarray, fallback_tol: float,
                        pool_factor: int = POOL_FACTOR):
    """Like skeleton.skeletonize, with rows drawn from the learned proposal.

    Returns (Skeletons, fallback flags per node).
    """
    from .skeleton import Skeletons, effective_samples
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
            out.nodes[a], fell[a] = skeletonize_learned_node(Xt, tree, a, cols, k, tol, max_rank, s, seed, theta,
                                                             mu, sd, fallback_tol, pool_factor)
    return out, fell


def skeletonize_learned_node(Xt, tree, a: int, cols: np.ndarray, k: Kernel, tol: float, max_rank: int, s: int,
                             seed: int, theta: np.ndarray, mu: np.ndarray, sd: np.ndarray, fallback_tol: float,
                             pool_factor: int = POOL_FACTOR):
    """One node of skeletonize_learned (tree-order points Xt, the node's columns given): (NodeSkeleton,
    whether it fell back to uniform rows)."""
    from .skeleton import NodeSkeleton, skeletonize_node
    b, e = int(tree.begin[a]), int(tree.end[a])
    if len(cols) > 0:
        pool = candidate_pool(b, e, tree.N, s, seed, a, pool_factor)
        geo = column_geometry(Xt[cols], seed, a)
        scores, _ = mlp_forward(theta, standardize(features(Xt[pool], geo), mu, sd))
        rows = select_rows(scores, pool, s, seed, a)
        Kp = kernel_matrix(Xt[rows], Xt[cols], k)
        idd = interpolative_decomposition(Kp, tol, max_rank)
        node = NodeSkeleton(cols=cols, rows=rows, rank=idd.rank, piv=idd.piv, skel=cols[idd.skel],
                            P=idd.P, rho=idd.rho, gap=idd.gap)
        if fallback_tol <= 0:
            return node, False
        hr = heldout_rows(b, e, tree.N, seed, a)
        Kh = kernel_matrix(Xt[hr], Xt[cols], k)
        if heldout_error(Kh, idd.skel, idd.P) <= fallback_tol:
            return node, False
        return skeletonize_node(Xt, tree, a, cols, k, tol, max_rank, s, seed), True
    return skeletonize_node(Xt, tree, a, cols, k, tol, max_rank, s, seed), False
