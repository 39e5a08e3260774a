"""Pins of the oracle's proposal training pieces: standardization, the epoch
visiting order, the training blocks and set, and mini-batch Adam.

Each test checks a property fixed by the definitions or by mathematics (closed
forms, permutations, invariants), not a re-typed formula.
"""
import math

import numpy as np
import pytest

from oracle import proposal as pr
from oracle.kernels import GAUSSIAN, Kernel
from oracle.tree import build_tree
from paper_1409_2802_amd import workloads as w


def test_fit_standardization_closed_form():
    F = np.zeros((4, pr.NF))
    F[:, 0] = [1.0, 2.0, 3.0, 4.0]          # mean 2.5, population variance 1.25
    F[:, 1] = 7.0                           # constant: sd floored
    F[:, 15] = 1.0
    mu, sd = pr.fit_standardization(F)
    assert mu[0] == 2.5 and sd[0] == pytest.approx(math.sqrt(1.25), rel=1e-15)
    assert mu[1] == 7.0 and sd[1] == 1e-6
    assert mu[15] == 0.0 and sd[15] == 1.0
    Z = pr.standardize(F, mu, sd)
    assert np.allclose(Z[:, 0].mean(), 0.0) and np.allclose(Z[:, 0].std(), 1.0)
    assert np.all(Z[:, 15] == 1.0)


@pytest.mark.parametrize("C", [1, 2, 7, 64, 96, 1000, 4096, 3 * 5 * 7 * 11])
def test_epoch_stride_gives_a_permutation(C):
    for e in range(6):
        k = pr.epoch_stride(C, 11, e)
        assert 1 <= k <= max(1, C - 1)
        order = (np.arange(C) * k) % C
        assert np.array_equal(np.sort(order), np.arange(C))


def test_adam_first_step_moves_every_parameter_by_lr():
    # Kingma & Ba: with bias correction the first update is lr * g / (|g| + eps),
    # i.e. lr in magnitude wherever |g| >> eps.
    rng = np.random.default_rng(0)
    F = rng.standard_normal((50, pr.NF))
    t = rng.standard_normal(50)
    theta0 = w.mlp_init(5)
    mu, sd = pr.fit_standardization(F)
    theta, _, _ = pr.train(F, t, theta0, epochs=1, batch=50, lr=1e-3, seed=0, mu=mu, sd=sd)
    _, g = pr.mlp_loss_grad(theta0, pr.standardize(F, mu, sd), t)
    big = np.abs(g) > 1e-5
    assert big.sum() > 1000
    assert np.allclose(np.abs(theta - theta0)[big], 1e-3, rtol=1e-2)
    assert np.array_equal(np.sign(theta0 - theta)[big], np.sign(g)[big])
    assert np.all(theta[g == 0.0] == theta0[g == 0.0])


def test_train_learns_a_smooth_target():
    rng = np.random.default_rng(1)
    F = rng.standard_normal((512, pr.NF))
    F[:, 15] = 1.0
    t = np.sin(F[:, 0]) + 0.5 * F[:, 1] * F[:, 2]
    mu, sd = pr.fit_standardization(F)
    theta, hist, steps = pr.train(F, t, w.mlp_init(5), epochs=40, batch=64, lr=3e-3, seed=2, mu=mu, sd=sd)
    assert len(hist) == 40 and len(steps) == 40 * 8
    assert hist[-1] < 0.25 * hist[0]
    # The epoch loss is the sample-weighted mean of the batch losses.
    assert hist[0] == pytest.approx(np.mean(steps[:8]), rel=1e-12)


def test_full_batch_epoch_is_one_gradient_step():
    rng = np.random.default_rng(3)
    F = rng.standard_normal((30, pr.NF))
    t = rng.standard_normal(30)
    mu, sd = pr.fit_standardization(F)
    th0 = w.mlp_init(5)
    theta, hist, _ = pr.train(F, t, th0, epochs=1, batch=1000, lr=1e-3, seed=0, mu=mu, sd=sd)
    # A permuted full batch has the same mean loss as the original order.
    loss, _ = pr.mlp_loss_grad(th0, pr.standardize(F, mu, sd), t)
    assert hist[0] == pytest.approx(loss, rel=1e-12)


def test_training_blocks_invariants():
    X = w.gaussian_mixture(3000, 6, k=8, seed=4)
    tree = build_tree(X, 200)
    blocks, n, m = pr.training_blocks(tree, 300, 150, 400, seed=9)
    leaves = list(tree.level_nodes(tree.depth))
    sizes = [int(tree.end[a] - tree.begin[a]) for a in leaves]
    assert n == min(150, min(sizes)) and m == min(400, tree.N - max(sizes))
    counts = np.zeros(len(leaves))
    for g, blk in enumerate(blocks):
        b, e = int(tree.begin[blk.leaf]), int(tree.end[blk.leaf])
        assert len(blk.cols) == n and len(np.unique(blk.cols)) == n
        assert np.all((blk.cols >= b) & (blk.cols < e))
        assert len(blk.rows) == m and len(np.unique(blk.rows)) == m
        assert np.all((blk.rows < b) | (blk.rows >= e)) and np.all((blk.rows >= 0) & (blk.rows < tree.N))
        assert np.all(np.diff(blk.cols) > 0) and np.all(np.diff(blk.rows) > 0)
        counts[blk.leaf - leaves[0]] += 1
    # Leaf choice is uniform: chi-square over 16 leaves, 300 draws (df 15; 0.1% point 37.7).
    exp = len(blocks) / len(leaves)
    assert ((counts - exp) ** 2 / exp).sum() < 37.7


def test_training_set_targets_are_normalized_log_leverage():
    X = w.low_intrinsic(1200, 8, di=3, seed=5)
    tree = build_tree(X, 150)
    k = Kernel(GAUSSIAN, h=1.0)
    F, lev, tgt, blocks = pr.training_set(X, tree, k, 5, 60, 200, eps=1e-3, seed=3)
    m = len(blocks[0].rows)
    assert F.shape == (5 * m, pr.NF) and np.all(F[:, 15] == 1.0)
    for g in range(5):
        l = lev[g * m:(g + 1) * m]
        assert np.all((l >= 0) & (l <= 1 + 1e-12))
        # exp(t) averages to 1 within a block when no leverage hits the floor.
        if l.min() > 1e-12:
            assert np.exp(tgt[g * m:(g + 1) * m]).mean() == pytest.approx(1.0, rel=1e-12)
