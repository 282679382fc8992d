"""Host-side comparison of switching orders (Sec. IV.D).

The paper compares the order in which magnets switch during a reversal in
two simulations by Spearman's rank correlation coefficient.  The flip logs
come from the device (asi_get_flip_log); ranking n magnets is O(n log n)
host work, so it stays on the host.
"""
from __future__ import annotations

import numpy as np


def switching_order(steps, idx, n: int) -> np.ndarray:
    """Position (0-based) of each magnet's first switch in a flip log of
    (step, index) pairs; magnets that never switch get position len(log)."""
    idx = np.asarray(idx, dtype=np.int64)
    pos = np.full(int(n), len(idx), dtype=np.int64)
    seen = np.zeros(int(n), dtype=bool)
    for k, j in enumerate(idx):
        if not seen[j]:
            seen[j] = True
            pos[j] = k
    return pos


def _average_ranks(x) -> np.ndarray:
    x = np.asarray(x)
    order = np.argsort(x, kind="stable")
    ranks = np.empty(len(x), dtype=np.float64)
    xs = x[order]
    start = 0
    while start < len(x):
        stop = start + 1
        while stop < len(x) and xs[stop] == xs[start]:
            stop += 1
        ranks[order[start:stop]] = 0.5 * (start + stop - 1) + 1.0   # ties share their mean rank
        start = stop
    return ranks


def spearman_rho(a, b) -> float:
    """Spearman's rank correlation of two equally long sequences: the Pearson
    correlation of their ranks, tied values taking the mean of their ranks."""
    ra, rb = _average_ranks(a), _average_ranks(b)
    if len(ra) != len(rb) or len(ra) < 2:
        raise ValueError("two sequences of the same length >= 2 are needed")
    da, db = ra - ra.mean(), rb - rb.mean()
    den = np.sqrt((da * da).sum() * (db * db).sum())
    return float((da * db).sum() / den) if den > 0 else float("nan")
