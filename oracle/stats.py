"""Oracle: Spearman rank correlation (Pearson correlation of average ranks).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Used to compare how
well fidelity orders string pairs by Levenshtein distance.
"""
from __future__ import annotations

import numpy as np


def average_ranks(x) -> np.ndarray:
    """Ranks 1..n; tied values share the mean of the ranks they span."""
    x = np.asarray(x, dtype=np.float64)
    order = np.argsort(x, kind="stable")
    xs = x[order]
    ranks = np.empty(x.shape[0], dtype=np.float64)
    i = 0
    n = x.shape[0]
    while i < n:
        j = i
        while j + 1 < n and xs[j + 1] == xs[i]:
            j += 1
        ranks[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return ranks


def pearson(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xc, yc = x - x.mean(), y - y.mean()
    return float(np.sum(xc * yc) / np.sqrt(np.sum(xc * xc) * np.sum(yc * yc)))


def spearman(x, y) -> float:
    return pearson(average_ranks(x), average_ranks(y))
