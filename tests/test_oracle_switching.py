"""Pins of the switching-order oracle (oracle/switching.py, Sec. IV.D).

P17: first-switch positions by hand; average ranks with ties by hand;
rho = 1 for one order against itself and -1 against its reverse; without
ties rho equals the textbook closed form 1 - 6 sum d^2 / (n (n^2 - 1));
with ties it equals scipy's spearmanr; and on the oracle's own runs the
switching order of a weakly coupled 4 x 4 square follows that of the same
array without coupling (the inherent order set by the coercive fields), while
strong coupling lowers the correlation.
"""
import math

import numpy as np
from scipy import stats

from oracle import native as N
from oracle import switching as S
from paper_2002_11401_amd import workloads as W


def test_p17_first_switch_positions_by_hand():
    assert S.first_switch_positions([3, 1, 3, 0], 5).tolist() == [3, 1, 4, 0, 4]
    assert S.first_switch_positions([], 3).tolist() == [0, 0, 0]
    assert S.first_switch_positions([2, 2, 2], 3).tolist() == [3, 3, 0]


def test_p17_average_ranks_by_hand():
    assert S.average_ranks([10, 20, 20, 30]).tolist() == [1.0, 2.5, 2.5, 4.0]
    assert S.average_ranks([5, 5, 5]).tolist() == [2.0, 2.0, 2.0]
    assert S.average_ranks([3, 1, 2]).tolist() == [3.0, 1.0, 2.0]
    # ranks always add up to n (n + 1) / 2
    x = np.random.default_rng(0).integers(0, 7, 101)
    assert S.average_ranks(x).sum() == 101 * 102 / 2


def test_p17_identical_and_reversed_orders():
    x = np.random.default_rng(1).permutation(500)
    assert S.spearman_rho(x, x)[0] == 1.0
    assert S.spearman_rho(x, -x)[0] == -1.0
    assert math.isnan(S.spearman_rho(np.ones(4), np.arange(4))[0])


def test_p17_closed_form_without_ties():
    rng = np.random.default_rng(2)
    for n in (2, 3, 17, 400):
        a, b = rng.permutation(n), rng.permutation(n)
        d = S.average_ranks(a) - S.average_ranks(b)
        closed = 1.0 - 6.0 * float((d * d).sum()) / (n * (n * n - 1))
        assert abs(S.spearman_rho(a, b)[0] - closed) < 1e-14


def test_p17_ties_match_scipy():
    rng = np.random.default_rng(3)
    for _ in range(6):
        a = rng.integers(0, 15, 60)
        b = a + rng.integers(-5, 6, 60)
        assert abs(S.spearman_rho(a, b)[0] - stats.spearmanr(a, b).statistic) < 1e-13
    # switching orders: never-switched magnets tie at the end
    pa = S.first_switch_positions([4, 0, 2, 4, 1], 6)
    pb = S.first_switch_positions([0, 1, 2, 3], 6)
    assert abs(S.spearman_rho(pa, pb)[0] - stats.spearmanr(pa, pb).statistic) < 1e-14


def test_p17_weak_coupling_follows_the_inherent_order():
    """4 x 4 closed square, b = 0.38, c = 1, beta = 1.5, gamma = 3.2, a
    reversal field increasing along 44 deg + 180 (Sec. IV.D): with weak
    coupling the switching order is that of the same array without
    coupling (set by h_k alone), so rho is close to 1; strong coupling
    lowers rho."""
    xy, theta = W.square_closed(4)
    n = len(theta)
    hk = W.disorder_hk(n, 0.2, 0.05, 9)
    H = W.linear_ramp(3000, 0.0, 0.3, 224.0)
    logs = {}
    for alpha in (0.0, 1e-5, 0.02):
        o = N.Oracle(xy, theta, hk, alpha, 10.0, 0.38, 1.0, 1.5, 3.2)
        o.set_spins(np.ones(n, np.int8))
        r = o.run(H)
        assert r["n_flips"] >= n
        logs[alpha] = r["idx"]
    inherent = S.first_switch_positions(logs[0.0], n)
    assert (inherent < len(logs[0.0])).all()          # every magnet reversed
    weak = S.switching_rho(logs[0.0], logs[1e-5], n)[0]
    strong = S.switching_rho(logs[0.0], logs[0.02], n)[0]
    assert weak > 0.95 and strong < weak
    # without coupling the order is the order of the switching fields, so it
    # correlates perfectly with it: magnets of one orientation switch in
    # ascending h_k
    horiz = theta == 0.0
    ph = inherent[horiz]
    assert S.spearman_rho(ph, hk[horiz])[0] == 1.0
