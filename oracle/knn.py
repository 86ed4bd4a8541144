"""Nearest-neighbour classification (k = 1) -- test infrastructure only.

The paper picks its sub-system size with a k-nearest-neighbours classifier fitted on
measured optima and finds k = 1 best (section "Building a heuristic for the optimum
sub-system size", the kNN paragraphs after Table I): a new size gets the label of the
closest measured size.  Here the same rule picks the tile G of the sweep for an (m, n) the
library has not timed.  This module states the rule plainly (distances to every training
point, the closest wins, ties to the earliest point) and the null accuracy the paper
compares against (always predicting the most frequent label).
"""
from __future__ import annotations

import numpy as np


def predict(train_x, train_y, x):
    """Label of the nearest training point (Euclidean distance) for every row of x; among
    equally near points the first in training order."""
    train_x = np.asarray(train_x, dtype=np.float64)
    train_y = np.asarray(train_y)
    x = np.asarray(x, dtype=np.float64)
    if train_x.ndim == 1:
        train_x = train_x[:, None]
    if x.ndim == 1:
        x = x[:, None]
    out = []
    for q in x:
        best, best_d = 0, np.inf
        for i, p in enumerate(train_x):
            d = float(np.sum((p - q) ** 2))
            if d < best_d:
                best, best_d = i, d
        out.append(train_y[best])
    return np.array(out)


# The paper's observed trend of the optimum sub-system size m over the system size N (section
# "Observations on the optimum sub-system size"): m is constant on each interval of N, the
# interval closed at its upper end.  Pairs (upper end of N, m).
_INTERVALS = ((4.5e3, 4), (2.5e4, 8), (5e4, 16), (7.5e4, 20), (1e7, 32), (1e8, 64))


def interval_rule(N) -> int:
    """The optimum m that the observed trend assigns to a system size N (0 < N <= 1e8)."""
    for upper, m in _INTERVALS:
        if N <= upper:
            return m
    raise ValueError("N beyond the sizes the trend covers")


def null_accuracy(y) -> float:
    """Accuracy of always predicting the most frequent label."""
    _, counts = np.unique(np.asarray(y), return_counts=True)
    return counts.max() / len(y)


def loo_accuracy(x, y) -> float:
    """Leave-one-out accuracy of the 1-NN rule."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y)
    hits = 0
    for i in range(len(y)):
        keep = np.arange(len(y)) != i
        hits += int(predict(x[keep], y[keep], x[i:i + 1])[0] == y[i])
    return hits / len(y)
