"""Input generators: lattice sizes and enumeration, protocols, seeding."""
import math

import numpy as np
import pytest

from oracle import native as N
from paper_2002_11401_amd import workloads as W


@pytest.mark.parametrize("side", [1, 4, 10, 100])
def test_square_counts_and_order(side):
    xy, theta = W.square_closed(side)
    nh = side * (side + 1)
    assert len(theta) == 2 * side * (side + 1)
    assert np.all(theta[:nh] == 0.0) and np.all(theta[nh:] == np.pi / 2)
    # horizontals: (x + 1/2, y), x fastest
    assert tuple(xy[0]) == (0.5, 0.0) and tuple(xy[side]) == (0.5, 1.0)
    if side > 1:
        assert tuple(xy[1]) == (1.5, 0.0)
    # verticals: (x, y + 1/2), x fastest
    assert tuple(xy[nh]) == (0.0, 0.5) and tuple(xy[nh + 1]) == (1.0, 0.5)
    # nearest-neighbour distance of the closed square lattice is sqrt(2)/2
    d = np.hypot(*(xy[:, None, :] - xy[None, :, :]).transpose(2, 0, 1)) if side <= 10 else None
    if d is not None:
        np.fill_diagonal(d, np.inf)
        assert abs(d.min() - math.sqrt(0.5)) < 1e-15


def test_pinwheel_is_square_rotated_by_45_degrees():
    xy, theta = W.square_closed(7)
    pxy, ptheta = W.pinwheel_diamond(7)
    assert np.array_equal(xy, pxy)
    assert np.allclose(ptheta - theta, np.pi / 4, atol=0, rtol=0)


def test_kagome_counts_angles_and_spacing():
    xy, theta = W.kagome(6)
    assert len(theta) == 3 * 36
    assert set(np.round(np.rad2deg(theta), 9)) == {30.0, 90.0, 150.0}
    d = np.hypot(*(xy[:, None, :] - xy[None, :, :]).transpose(2, 0, 1))
    np.fill_diagonal(d, np.inf)
    # islands at bond midpoints of a honeycomb with edge 1: nearest sqrt(3)/2
    assert abs(d.min() - math.sqrt(3) / 2) < 1e-12
    # every island axis lies along the bond it sits on: the two vertices of
    # the bond are at +-1/2 along the axis, and each vertex joins 3 bonds
    ends = np.concatenate([xy + 0.5 * np.stack([np.cos(theta), np.sin(theta)], 1),
                           xy - 0.5 * np.stack([np.cos(theta), np.sin(theta)], 1)])
    keys = np.round(ends, 6)
    _, counts = np.unique(keys, axis=0, return_counts=True)
    assert counts.max() == 3


def test_kagome_1m_size_and_neighbour_count():
    assert 3 * 577 * 577 == 998787
    xy, theta = W.kagome(40)
    o = N.Oracle(xy, theta, np.full(len(theta), 0.15), 0.002, 3.0, 1, 1, 3, 3)
    deg = np.diff(o.neighbours()[0])
    assert deg.max() == 32   # interior kagome island, neighbour distance 3


def test_protocols():
    H = W.triangle_ramp(100, 0.3, 45.0)
    assert H.shape == (200, 2)
    assert np.allclose(H[0], [0.3 * math.cos(math.pi / 4), 0.3 * math.sin(math.pi / 4)])
    assert np.allclose(H[99], -H[0]) and np.allclose(H[199], H[0])
    R = W.rotating(2000, 0.08, 1000)
    assert np.allclose(np.hypot(R[:, 0], R[:, 1]), 0.08)
    assert np.allclose(R[1000], R[0])
    L = W.linear_ramp(2000, 0.1, -0.1, 30.0)
    assert np.allclose(L[0], [0.1 * math.cos(math.pi / 6), 0.1 * math.sin(math.pi / 6)])


def test_disorder_is_seeded_positive_and_has_the_stated_moments():
    a = W.disorder_hk(200000, 0.2, 0.05, 7)
    b = W.disorder_hk(200000, 0.2, 0.05, 7)
    assert np.array_equal(a, b)
    assert np.all(a > 0)
    assert abs(a.mean() - 0.2) < 1e-4 and abs(a.std() - 0.01) < 1e-4
    assert not np.array_equal(a, W.disorder_hk(200000, 0.2, 0.05, 8))


def test_polarised_spins():
    theta = np.array([0.0, np.pi / 2, np.pi, 3 * np.pi / 4])
    s = W.polarised_spins(theta, [1.0, 0.0])
    assert s.tolist() == [1, 1, -1, -1]   # cos(pi/2) rounds to +6e-17 >= 0
    assert W.square_10x10_triangle().spin0.tolist() == [1] * 220


def test_named_workloads_shapes():
    w = W.square_10x10_triangle()
    assert (w.n, w.n_steps) == (220, 200)
    w = W.pinwheel_100x100_reversal()
    assert (w.n, w.n_steps) == (20200, 2000)


def test_sweep_and_stream_are_reproducible_and_in_range():
    a = W.batched_sweep(count=40, seed=4, n_steps=10)
    b = W.batched_sweep(count=40, seed=4, n_steps=10)
    assert [w.name for w in a] == [w.name for w in b]
    for w in a:
        assert 840 <= w.n <= 80400 and w.neighbor_distance in (1.0, 3.0, 10.0)
        assert w.H.shape == (10, 2)
    jobs = W.served_stream(count=300, seed=5)
    arr = np.array([j.arrival_s for j in jobs])
    assert np.all(np.diff(arr) > 0)
    rate = len(jobs) / arr[-1]
    assert 35 < rate < 70
    assert all(1e3 <= j.n_target <= 1e6 and 1 <= j.d <= 10 and 100 <= j.n_steps <= 2000
               for j in jobs)
    w = jobs[3].workload()
    assert abs(w.n - jobs[3].n_target) / jobs[3].n_target < 0.1


def _min_separation(xy):
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    return d.min()


def test_open_square_lucky_knot_and_ising():
    n = 7
    xy, theta = W.square_open(n)
    assert len(theta) == 2 * n * (n - 1)
    closed, _ = W.square_closed(n)
    assert {tuple(p) for p in xy} < {tuple(p) for p in closed}
    # no island on the outer boundary: every vertex of the outline is open
    assert xy[:, 0].min() > 0 and xy[:, 1].min() > 0 and xy[:, 0].max() < n and xy[:, 1].max() < n
    xy, theta = W.pinwheel_lucky_knot(12)
    assert set(np.round(np.degrees(theta)).astype(int)) == {0, 90}
    assert xy.min() >= 0.0 and xy.max() <= 12.0
    assert abs(_min_separation(xy) - np.sqrt(0.5)) < 1e-12
    # the lattice is turned by 45 deg: an island's four nearest neighbours
    # (the diagonal ones of the square lattice) now lie along the x and y axes
    i = int(np.argmin(((xy - 6.0) ** 2).sum(1)))
    d = xy - xy[i]
    r = np.hypot(d[:, 0], d[:, 1])
    near = d[(r > 0) & (r < np.sqrt(0.5) + 1e-9)]
    assert len(near) == 4 and np.allclose(near[:, 0] * near[:, 1], 0.0, atol=1e-15)
    xy, theta = W.ising(5, 3)
    assert len(theta) == 15 and not theta.any() and _min_separation(xy) == 1.0


def test_local_field_and_schedule_generators():
    xy, _ = W.kagome(4)
    g = W.spatial_gradient(xy, 0.01, 90.0, 0.0)
    assert g.shape == (len(xy), 2) and np.allclose(g[:, 0], 0.0, atol=1e-15)
    assert abs(g[:, 1].sum()) < 1e-12          # measured from the centre
    wv = W.travelling_wave(xy, 5, 0.1, 3.0, 4, 0.0)
    assert wv.shape == (5, len(xy), 2) and np.abs(wv).max() <= 0.1
    assert np.allclose(wv[4], W.travelling_wave(xy, 1, 0.1, 3.0, 4, 0.0)[0])  # period 4 steps
    s = W.exponential_anneal(11, 0.2, 0.002)
    assert s[0] == 0.2 and abs(s[-1] - 0.002) < 1e-15 and np.allclose(s[1:] / s[:-1], 0.01 ** 0.1)


def test_square_vertices_groups():
    n = 5
    xy, theta = W.square_closed(n)
    ptr, idx, vxy = W.square_vertices(n)
    assert len(ptr) == (n + 1) ** 2 + 1 and ptr[-1] == len(idx) == 2 * len(theta)
    for g in range(len(ptr) - 1):
        members = idx[ptr[g]:ptr[g + 1]]
        assert np.allclose(np.hypot(*(xy[members] - vxy[g]).T), 0.5)
        inner = 0 < vxy[g, 0] < n and 0 < vxy[g, 1] < n
        assert len(members) == (4 if inner else len(members)) and 2 <= len(members) <= 4


def test_sinusoidal_and_sawtooth_protocols():
    H = W.sinusoidal(40, 0.1, 20, 30.0)
    assert H.shape == (40, 2)
    strength = H @ np.array([np.cos(np.radians(30)), np.sin(np.radians(30))])
    assert abs(strength[5] - 0.1) < 1e-15 and abs(strength[15] + 0.1) < 1e-15
    assert np.allclose(strength[:20], strength[20:])
    S = W.sawtooth(25, 0.2, 5, 0.0)
    assert np.allclose(S[:, 1], 0.0)
    assert S[0, 0] == -0.2 and S[4, 0] == 0.2 and S[5, 0] == -0.2
    assert np.all(np.diff(S[:5, 0]) > 0)
