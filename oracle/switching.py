"""Oracle: comparison of switching orders by Spearman's rank correlation.

TEST INFRASTRUCTURE ONLY: imported by tests/ alone; the product path never
imports it, and it shares no code with the HIP library.

Sec. IV.D of the paper compares the order in which the magnets of an array
switch during a reversal in two simulations, by Spearman's rank correlation
coefficient rho: 1 for the same order, 0 for unrelated orders.  Written out
as the definition, in three steps:

  1. switching order: the position, in a flip log of (step, magnet) pairs,
     of each magnet's first switch; a magnet that never switches is placed
     after every switch (position = length of the log), so such magnets tie;
  2. ranks: each value's rank among the n values (1 = smallest), tied values
     sharing the mean of the ranks they occupy;
  3. rho: Pearson's correlation coefficient of the two rank vectors.

Step 3 is evaluated exactly: average ranks are multiples of 1/2 and their
mean is (n + 1) / 2, so u = 2 r - (n + 1) is an integer vector with the same
correlation; the three sums of products of u are formed as Python integers,
and rho = Sab / sqrt(Saa * Sbb) with each integer rounded to the nearest
double first.  rho is NaN when either order has all values tied.
"""
from __future__ import annotations

import math

import numpy as np


def first_switch_positions(idx, n: int) -> np.ndarray:
    """Step 1: position of each magnet's first entry in the flip log
    (magnet indices `idx` in log order); len(idx) for magnets absent."""
    L = len(idx)
    pos = np.full(int(n), L, dtype=np.int64)
    for k, j in enumerate(np.asarray(idx, dtype=np.int64).tolist()):
        if pos[j] == L:
            pos[j] = k
    return pos


def average_ranks(x) -> np.ndarray:
    """Step 2: rank of each value among all values, 1 for the smallest; a
    group of equal values occupying ranks s .. e gets (s + e) / 2 each."""
    x = np.asarray(x)
    order = np.argsort(x, kind="stable")
    xs = x[order]
    ranks = np.empty(len(x), dtype=np.float64)
    s = 0
    while s < len(x):
        e = s
        while e + 1 < len(x) and xs[e + 1] == xs[s]:
            e += 1
        ranks[order[s:e + 1]] = 0.5 * ((s + 1) + (e + 1))
        s = e + 1
    return ranks


def rank_sums(ra, rb):
    """Exact sums (Sab, Saa, Sbb) of u_a u_b, u_a^2 and u_b^2 over the
    magnets, u = 2 r - (n + 1) for average ranks r (integers)."""
    n = len(ra)
    ua = [int(round(2.0 * v)) - (n + 1) for v in np.asarray(ra).tolist()]
    ub = [int(round(2.0 * v)) - (n + 1) for v in np.asarray(rb).tolist()]
    return (sum(p * q for p, q in zip(ua, ub)), sum(p * p for p in ua),
            sum(q * q for q in ub))


def spearman_rho(a, b):
    """Spearman's rho of two equally long value sequences (steps 2 and 3):
    returns (rho, (Sab, Saa, Sbb))."""
    if len(a) != len(b) or len(a) < 2:
        raise ValueError("two sequences of the same length >= 2 are needed")
    sab, saa, sbb = rank_sums(average_ranks(a), average_ranks(b))
    den = math.sqrt(float(saa) * float(sbb))
    rho = float(sab) / den if den > 0.0 else float("nan")
    return rho, (sab, saa, sbb)


def switching_rho(idx_a, idx_b, n: int):
    """rho of the switching orders of two flip logs of the same n magnets."""
    return spearman_rho(first_switch_positions(idx_a, n), first_switch_positions(idx_b, n))
