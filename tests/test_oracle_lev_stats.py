"""Pins of the Levenshtein and Spearman oracles."""
import itertools

import numpy as np
import pytest
import scipy.stats

from oracle import lev, stats
from synth import mutate_pairs


def test_levenshtein_matches_bfs_on_all_tiny_pairs():
    alpha = (0, 1, 2)
    strings = [s for n in range(0, 4) for s in itertools.product(alpha, repeat=n)]
    rng = np.random.default_rng(0)
    pick = rng.choice(len(strings), size=(120, 2))
    for i, j in pick:
        a, b = strings[i], strings[j]
        assert lev.levenshtein(a, b) == lev.levenshtein_brute(a, b, alpha)


def test_levenshtein_textbook_properties():
    rng = np.random.default_rng(1)
    for _ in range(50):
        a = rng.integers(0, 4, rng.integers(0, 12))
        b = rng.integers(0, 4, rng.integers(0, 12))
        c = rng.integers(0, 4, rng.integers(0, 12))
        assert lev.levenshtein(a, a) == 0
        assert lev.levenshtein(a, []) == len(a)
        assert lev.levenshtein(a, b) == lev.levenshtein(b, a)
        assert lev.levenshtein(a, c) <= lev.levenshtein(a, b) + lev.levenshtein(b, c)
        if len(a) == len(b):
            assert lev.levenshtein(a, b) <= int(np.sum(a != b))
    assert lev.levenshtein([0, 1, 2, 3], [1, 2, 3]) == 1       # one deletion
    assert lev.levenshtein([0, 0, 0], [1, 1, 1]) == 3          # three substitutions


def test_c_dp_matches_python_dp_and_edit_counts():
    p = mutate_pairs(300, 40, 12, seed=5)
    d = lev.lev_many(p.a, p.a_off, p.b, p.b_off)
    for i in range(p.n):
        a, b = p.pair(i)
        assert d[i] == lev.levenshtein(a, b)
    assert np.all(d <= p.edits)       # LD never exceeds the number of edits applied
    assert np.all(d >= np.abs(np.diff(p.b_off) - 40))


def test_spearman_matches_scipy_with_ties():
    rng = np.random.default_rng(2)
    for _ in range(10):
        x = rng.integers(0, 8, 200).astype(float)
        y = x + rng.normal(0, 3, 200)
        y[::7] = np.round(y[::7])
        assert abs(stats.spearman(x, y) - scipy.stats.spearmanr(x, y).statistic) < 1e-12
    x = rng.normal(size=50)
    assert abs(stats.spearman(x, np.exp(x)) - 1) < 1e-12      # monotone transform
    assert abs(stats.spearman(x, -x) + 1) < 1e-12
    assert np.allclose(stats.average_ranks([3, 1, 3, 2]), [3.5, 1, 3.5, 2])
