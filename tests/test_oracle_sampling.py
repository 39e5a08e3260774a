"""Pins for the oracle's uniform row sampler (Section 4.1.3, uniform sampling
without replacement; SplitMix64 and Floyd's algorithm from their publications)."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle.sampling import counter_u64, floyd_sample, sample_far_rows, splitmix64_next


def test_splitmix64_published_sequence():
    # First outputs of SplitMix64 seeded with 1234567, as listed with the
    # generator's public-domain reference implementation.
    expected = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                4593380528125082431, 16408922859458223821]
    s, got = 1234567, []
    for _ in expected:
        s, o = splitmix64_next(s)
        got.append(o)
    assert got == expected


def test_counter_generator_is_a_function_of_its_counter():
    assert counter_u64(7, 3, 11) == counter_u64(7, 3, 11)
    assert len({counter_u64(7, 3, j) for j in range(1000)}) == 1000
    assert counter_u64(7, 3, 11) != counter_u64(7, 4, 11)


@pytest.mark.parametrize("M,s", [(10, 3), (1792, 128), (100, 99), (5, 5), (4, 9), (1, 1)])
def test_floyd_distinct_sorted_in_range(M, s):
    out = floyd_sample(M, s, seed=3, stream=2)
    assert len(out) == min(M, s)
    assert out == sorted(set(out))
    assert all(0 <= t < M for t in out)


def test_far_rows_exclude_the_node():
    rows = sample_far_rows(b=100, e=300, N=1000, s=500, seed=1, node=9)
    assert len(rows) == 500 and len(set(rows.tolist())) == 500
    assert not np.any((rows >= 100) & (rows < 300))
    assert rows.min() >= 0 and rows.max() < 1000
    everything = sample_far_rows(b=100, e=300, N=1000, s=10_000, seed=1, node=9)
    assert everything.tolist() == list(range(100)) + list(range(300, 1000))


def test_floyd_subsets_are_uniform():
    """All C(5,2) = 10 subsets appear with equal frequency (chi-square)."""
    counts = {c: 0 for c in itertools.combinations(range(5), 2)}
    trials = 20000
    for seed in range(trials):
        counts[tuple(floyd_sample(5, 2, seed=seed, stream=0))] += 1
    chi2 = stats.chisquare(list(counts.values()))
    assert chi2.pvalue > 1e-4


def test_inclusion_frequency_is_s_over_m():
    M, s, trials = 40, 7, 6000
    hits = np.zeros(M)
    for seed in range(trials):
        hits[floyd_sample(M, s, seed=seed, stream=5)] += 1
    chi2 = stats.chisquare(hits, np.full(M, trials * s / M))
    assert chi2.pvalue > 1e-4
