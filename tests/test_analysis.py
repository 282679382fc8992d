"""Switching-order comparison (Sec. IV.D) on the host."""
import numpy as np
from scipy import stats

from oracle import native as N
from paper_2002_11401_amd import analysis as A
from paper_2002_11401_amd import workloads as W


def test_spearman_matches_scipy_with_ties():
    rng = np.random.default_rng(1)
    for _ in range(5):
        a = rng.integers(0, 15, 40)
        b = a + rng.integers(-4, 5, 40)
        assert abs(A.spearman_rho(a, b) - stats.spearmanr(a, b).statistic) < 1e-12
    x = np.arange(10)
    assert A.spearman_rho(x, x) == 1.0 and A.spearman_rho(x, -x) == -1.0


def test_switching_order_positions():
    pos = A.switching_order([0, 0, 1, 1], [3, 1, 3, 0], 5)
    assert pos.tolist() == [3, 1, 4, 0, 4]


def test_weak_coupling_order_follows_the_coercive_fields():
    """A weakly coupled 4 x 4 closed square under a reversal field along the
    diagonal switches in the order of its coercive fields (Sec. IV.D), so
    the order's rank correlation with h_k is close to 1; strong coupling
    lowers it."""
    xy, theta = W.square_closed(4)
    n = len(theta)
    hk = W.disorder_hk(n, 0.2, 0.05, 9)
    H = W.linear_ramp(2000, 0.0, 0.3, 225.0)     # against both sublattices
    rhos = []
    for alpha in (1e-5, 0.02):
        o = N.Oracle(xy, theta, hk, alpha, 10.0, 0.38, 1.0, 1.5, 3.2)
        o.set_spins(np.ones(n, np.int8))
        r = o.run(H)
        pos = A.switching_order(r["step"], r["idx"], n)
        assert (pos < len(r["idx"])).all()          # everything reversed
        rhos.append(A.spearman_rho(pos, hk))
    assert rhos[0] > 0.95 and rhos[1] < rhos[0]
