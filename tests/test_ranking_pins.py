"""Pins of the Monte-Carlo ranking oracle (Sec. "Monte-Carlo Ranking",
Table 2): SplitMix64's published outputs, a worked example derived from
them by hand, and properties that any correct ranking has."""
import math

import numpy as np
import pytest

from oracle import ranking


def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 started at state 0
    st, a = ranking.splitmix64(0)
    st, b = ranking.splitmix64(st)
    st, c = ranking.splitmix64(st)
    assert (a, b, c) == (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F)


def test_worked_example():
    # n = 10, seed 0, S = 3: h/2^64 = 0.883.., 0.431.., 0.026.. pick
    # individuals 8, 4 and 0.  Fitness = 0..9, lower is better, so the
    # sampled values are 8, 4, 0.
    assert ranking.sample_indices(10, 0, 3) == [8, 4, 0]
    band, children, sample = ranking.mc_rank(np.arange(10.0), False, 0, S=3)
    # value 3 beats 8 and 4: 2 of 3 -> percentile 66 -> band 60 (1 child);
    # value 0 ties with the sampled 0: still 2 -> 60; value 5 beats 8 only:
    # 33 -> 30 (0.15); value 9 beats none: 0 (0.01)
    assert band[3] == 60 and band[0] == 60 and band[5] == 30 and band[9] == 0
    assert children[3] == pytest.approx(1.0) and children[5] == pytest.approx(0.15)
    assert children[9] == pytest.approx(0.01)
    assert list(sample) == [-8.0, -4.0, -0.0]


def test_table2_keeps_population_size_on_average():
    # the ten bands' expected children sum to 10: a representative sample
    # keeps the population size
    assert math.isclose(sum(ranking.CHILDREN.values()), 10.0)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(100_000)
    means = [ranking.mc_rank(f, False, seed, S=100)[1].mean() for seed in range(8)]
    assert 0.85 < np.mean(means) < 1.15


def test_ties_and_invalid_values():
    # equal fitness: nobody beats anybody
    band, _, _ = ranking.mc_rank(np.full(500, 2.5), False, 7)
    assert (band == 0).all()
    # NaN is the worst value, both as an individual and in the sample
    f = np.array([np.nan, 1.0, 2.0, np.nan, np.inf])
    band, _, sample = ranking.mc_rank(f, False, 3, S=50)
    assert band[0] == 0 and band[3] == 0
    assert band[1] >= band[2] >= band[4]


def test_direction_symmetry_and_monotonicity():
    rng = np.random.default_rng(9)
    f = rng.uniform(-5, 5, 3000)
    b1, c1, s1 = ranking.mc_rank(f, False, 11)
    b2, c2, s2 = ranking.mc_rank(-f, True, 11)
    assert np.array_equal(b1, b2) and np.array_equal(c1, c2) and np.array_equal(s1, s2)
    order = np.argsort(f)                 # best (lowest) first
    assert np.all(np.diff(b1[order]) <= 0)
