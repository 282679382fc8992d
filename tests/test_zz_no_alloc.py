"""The allocation-free switching-order comparison (asi_switching_rho_noalloc)
against the allocating one (asi_switching_rho) and the oracle, through the
C ABI: the same rho and exact rank sums, bit for bit, on two calls in a row
(the second on a smaller instance, so it runs over what the first left in
the static scratch), and its size limit.
"""
import sys

import numpy as np
import pytest

from oracle import native as N
from oracle import switching as S
from paper_2002_11401_amd import asi
from paper_2002_11401_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def run_pair(pair):
    sims, logs = [], []
    for w in pair:
        sim = asi.Sim.from_workload(w)
        sim.run()
        o = N.Oracle.from_workload(w)
        o.set_spins(w.spin0)
        r = o.run(w.H, log_cap=10 ** 7)
        o.close()
        assert not r["truncated"]
        sims.append(sim)
        logs.append(r["idx"])
    return sims, logs


def kagome_pair():
    kxy, kth = W.kagome(80)
    kH = W.rotating(400, 0.08, 400)[:230]
    return [W.Workload(f"kagome80_seed{sd}", kxy, kth, W.polarised_spins(kth, kH[0]),
                       W.disorder_hk(len(kth), 0.15, 0.05, 2), kH, alpha=0.002,
                       neighbor_distance=3.0, b=1, c=1, beta=3, gamma=3, thermal_std=0.005,
                       thermal_seed=sd) for sd in (2, 3)]


def square_pair():
    xy, theta = W.square_closed(4)
    n = len(theta)
    hk = W.disorder_hk(n, 0.2, 0.05, 9)
    H = W.linear_ramp(3000, 0.0, 0.3, 224.0)
    return [W.Workload(f"square4_a{alpha}", xy, theta, np.ones(n, np.int8), hk, H, alpha=alpha,
                       neighbor_distance=10.0, b=0.38, c=1.0, beta=1.5, gamma=3.2)
            for alpha in (0.0, 0.02)]


def test_noalloc_rho_equals_allocating_rho_twice():
    for label, pair in (("kagome80 (19,200 magnets)", kagome_pair()),
                        ("square4 (40 magnets)", square_pair())):
        say("noalloc rho", label)
        sims, logs = run_pair(pair)
        n = pair[0].n
        ref = asi.switching_rho(sims[0], sims[1])
        got = asi.switching_rho_noalloc(sims[0], sims[1])
        want = S.switching_rho(logs[0], logs[1], n)
        say("rho", got, "allocating", ref, "oracle", want)
        assert got[1] == ref[1] == want[1]
        assert got[0] == ref[0] == want[0]
        # one instance against itself: rho = 1 through the shared path
        assert asi.switching_rho_noalloc(sims[1], sims[1]) == asi.switching_rho(sims[1], sims[1])
        for s in sims:
            s.close()


def test_noalloc_rho_rejects_sizes_beyond_its_limit():
    xy, theta = W.square_closed(725)  # 1,052,700 magnets > 2^20
    n = len(theta)
    say("noalloc rho limit", n)
    w = W.Workload("square725", xy, theta, np.ones(n, np.int8), np.full(n, 0.2),
                   W.linear_ramp(2, 0.0, 0.0, 0.0), alpha=0.001, neighbor_distance=1.0, b=1,
                   c=1, beta=3, gamma=3)
    sim = asi.Sim.from_workload(w)
    sim.run()
    with pytest.raises(asi.AsiError) as e:
        asi.switching_rho_noalloc(sim, sim)
    assert "2^20" in str(e.value)
    # no magnet switched: every rank ties, rho is NaN on the allocating path
    assert np.isnan(asi.switching_rho(sim, sim)[0])
    sim.close()
