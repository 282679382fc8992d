"""Seeded synthetic inputs shaped like the flatspin paper's workloads.

This module only *generates inputs*: magnet positions and rotations for the
standard geometries (paper Sec. II.I, Fig. 3), explicit external-field time
series (Sec. II.D), coercive-field disorder draws (Sec. II.G) and start
spins.  It contains none of the model's arithmetic (no dipolar field, no
switching astroid, no relaxation), so both the HIP path and the CPU oracle can
consume the very same arrays without sharing any computation.

Geometry readings (the paper only pictures the lattices):
  * square, closed edges: N x N vertex cells, lattice spacing 1; horizontal
    islands at (x+1/2, y), y = 0..N, x = 0..N-1 (angle 0), then vertical
    islands at (x, y+1/2), y = 0..N-1, x = 0..N (angle 90 deg); 2N(N+1)
    magnets, enumerated in exactly that order.
  * pinwheel "diamond": the square positions with every island rotated by
    45 deg about its centre (Sec. IV.C), i.e. angles 45 and 135 deg.
  * kagome: islands on the edges of a honeycomb whose edge length is 1.
    Y-shaped vertices sit on a triangular lattice
    (sqrt3*u + sqrt3/2*(v mod 2), 1.5*v); each owns the three half-bonds
    at (0, 1/2) angle 90, (-sqrt3/4, -1/4) angle 30 and (sqrt3/4, -1/4) angle
    150; enumeration is v-major, then u, then those three.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

SQRT3 = math.sqrt(3.0)


# --------------------------------------------------------------------------
# geometries (Sec. II.I)
# --------------------------------------------------------------------------

def square_closed(n_side: int):
    """Square ASI with closed edges: returns (xy[n,2], theta[n]) float64."""
    n = int(n_side)
    if n < 1:
        raise ValueError("n_side must be >= 1")
    yh, xh = np.meshgrid(np.arange(n + 1, dtype=np.float64),
                         np.arange(n, dtype=np.float64), indexing="ij")
    horiz = np.stack([xh.ravel() + 0.5, yh.ravel()], axis=1)
    yv, xv = np.meshgrid(np.arange(n, dtype=np.float64),
                         np.arange(n + 1, dtype=np.float64), indexing="ij")
    vert = np.stack([xv.ravel(), yv.ravel() + 0.5], axis=1)
    xy = np.ascontiguousarray(np.concatenate([horiz, vert], axis=0))
    theta = np.concatenate([np.zeros(len(horiz)),
                            np.full(len(vert), np.pi / 2)])
    return xy, np.ascontiguousarray(theta)


def pinwheel_diamond(n_side: int):
    """Pinwheel "diamond": square positions, every island turned by 45 deg."""
    xy, theta = square_closed(n_side)
    return xy, np.ascontiguousarray(theta + np.pi / 4)


def square_open(n_side: int):
    """Square ASI with open edges: the closed n_side x n_side lattice without
    its boundary ring of islands (horizontals on rows 1..n-1, verticals on
    columns 1..n-1), so the outer vertices are left open; 2n(n-1) magnets,
    horizontals first."""
    xy, theta = square_closed(n_side)
    n = int(n_side)
    keep = np.where(theta == 0.0, (xy[:, 1] > 0) & (xy[:, 1] < n), (xy[:, 0] > 0) & (xy[:, 0] < n))
    return np.ascontiguousarray(xy[keep]), np.ascontiguousarray(theta[keep])


def pinwheel_lucky_knot(n_side: int):
    """Pinwheel "lucky-knot": the pinwheel lattice (islands turned 45 deg)
    with the whole lattice turned a further 45 deg, so the array's outline
    runs along the lattice diagonals; cut to the square of side n_side
    (lattice units) centred on a vertex.  Islands then lie at 0 and 90 deg.
    Ordered by y, then x."""
    n = int(n_side)
    m = int(math.ceil(n * math.sqrt(2.0))) + 2
    xy, theta = square_closed(2 * m)
    xy = xy - float(m)
    c = math.sqrt(0.5)
    rot = np.stack([c * xy[:, 0] - c * xy[:, 1], c * xy[:, 0] + c * xy[:, 1]], axis=1)
    ang = np.mod(theta + np.pi / 2, np.pi)
    half = n / 2.0
    keep = (np.abs(rot[:, 0]) <= half) & (np.abs(rot[:, 1]) <= half)
    rot, ang = rot[keep] + half, ang[keep]
    order = np.lexsort((rot[:, 0], rot[:, 1]))
    return np.ascontiguousarray(rot[order]), np.ascontiguousarray(ang[order])


def ising(nx: int, ny: Optional[int] = None):
    """Ising ASI: islands on a square grid of spacing 1, all along x (one
    sublattice); nx * ny magnets, row-major."""
    ny = nx if ny is None else ny
    yy, xx = np.meshgrid(np.arange(int(ny), dtype=np.float64),
                         np.arange(int(nx), dtype=np.float64), indexing="ij")
    xy = np.stack([xx.ravel(), yy.ravel()], axis=1)
    return np.ascontiguousarray(xy), np.zeros(len(xy))


def square_vertices(n_side: int):
    """The islands meeting at each vertex (x, y) of square_closed(n_side),
    vertices row-major, islands in index order: (ptr [V+1], idx, vxy [V,2])."""
    n = int(n_side)
    xy, theta = square_closed(n)
    nh = n * (n + 1)
    ptr, idx, vxy = [0], [], []
    for y in range(n + 1):
        for x in range(n + 1):
            members = []
            if x > 0:
                members.append(y * n + (x - 1))          # horizontal to the left
            if x < n:
                members.append(y * n + x)                # horizontal to the right
            if y > 0:
                members.append(nh + (y - 1) * (n + 1) + x)   # vertical below
            if y < n:
                members.append(nh + y * (n + 1) + x)         # vertical above
            idx.extend(sorted(members))
            ptr.append(len(idx))
            vxy.append((float(x), float(y)))
    return (np.asarray(ptr, dtype=np.int64), np.asarray(idx, dtype=np.int32),
            np.asarray(vxy, dtype=np.float64))


def kagome(nu: int, nv: Optional[int] = None):
    """Kagome ASI on nu x nv honeycomb cells (3 islands per cell)."""
    nu = int(nu)
    nv = nu if nv is None else int(nv)
    if nu < 1 or nv < 1:
        raise ValueError("kagome needs nu, nv >= 1")
    v, u = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    ox = SQRT3 * u + (SQRT3 / 2.0) * (v % 2)
    oy = 1.5 * v
    ox = ox.ravel().astype(np.float64)
    oy = oy.ravel().astype(np.float64)
    offs = np.array([[0.0, 0.5], [-SQRT3 / 4.0, -0.25], [SQRT3 / 4.0, -0.25]])
    angs = np.array([np.pi / 2, np.pi / 6, 5 * np.pi / 6])
    x = (ox[:, None] + offs[None, :, 0]).ravel()
    y = (oy[:, None] + offs[None, :, 1]).ravel()
    xy = np.ascontiguousarray(np.stack([x, y], axis=1))
    theta = np.ascontiguousarray(np.tile(angs, len(ox)))
    return xy, theta


def kagome_cells_for(n_target: int) -> int:
    """Square cell count nu (= nv) whose kagome patch is closest to n_target."""
    return max(1, int(round(math.sqrt(n_target / 3.0))))


def square_side_for(n_target: int) -> int:
    """Side N whose closed square lattice 2N(N+1) is closest to n_target."""
    return max(1, int(round((-1.0 + math.sqrt(1.0 + 2.0 * n_target)) / 2.0)))


GEOMETRIES = {"square": square_closed, "pinwheel": pinwheel_diamond,
              "kagome": kagome}


# --------------------------------------------------------------------------
# external-field protocols (Sec. II.D): explicit arrays H[t] = (hx, hy)
# --------------------------------------------------------------------------

def _along(h: np.ndarray, angle_deg: float) -> np.ndarray:
    a = np.deg2rad(angle_deg)
    return np.ascontiguousarray(np.stack([h * np.cos(a), h * np.sin(a)], axis=1))


def linear_ramp(n_steps: int, h0: float, h1: float, angle_deg: float):
    """Field of strength linspace(h0, h1, n_steps) along a fixed angle."""
    return _along(np.linspace(h0, h1, int(n_steps)), angle_deg)


def triangle_ramp(half_steps: int, amp: float, angle_deg: float):
    """+amp -> -amp in half_steps points, then -amp -> +amp in half_steps."""
    down = np.linspace(amp, -amp, int(half_steps))
    up = np.linspace(-amp, amp, int(half_steps))
    return _along(np.concatenate([down, up]), angle_deg)


def sinusoidal(n_steps: int, amp: float, steps_per_period: float, angle_deg: float,
               phase_deg: float = 0.0):
    """Field amp * sin(2 pi t / steps_per_period + phase) along a fixed angle."""
    t = np.arange(int(n_steps), dtype=np.float64)
    return _along(amp * np.sin(2.0 * np.pi * t / float(steps_per_period) + np.deg2rad(phase_deg)),
                  angle_deg)


def sawtooth(n_steps: int, amp: float, steps_per_period: int, angle_deg: float):
    """Field rising linearly from -amp to +amp over each period, then
    dropping back: amp * (2 (t mod P) / (P - 1) - 1) along a fixed angle."""
    P = int(steps_per_period)
    t = np.arange(int(n_steps)) % P
    return _along(amp * (2.0 * t / max(1, P - 1) - 1.0), angle_deg)


def rotating(n_steps: int, amp: float, steps_per_rev: int, phase_deg: float = 0.0):
    """Field of fixed strength whose angle advances 2*pi/steps_per_rev per step."""
    t = np.arange(int(n_steps), dtype=np.float64)
    phi = 2.0 * np.pi * t / float(steps_per_rev) + np.deg2rad(phase_deg)
    return np.ascontiguousarray(np.stack([amp * np.cos(phi), amp * np.sin(phi)], axis=1))


# per-magnet (local and spatial) fields, Sec. II.D: arrays h_loc[i] or
# h_loc[t][i], added to the global H[t] by the model
def spatial_gradient(xy: np.ndarray, grad: float, angle_deg: float, axis_deg: float = 0.0):
    """Static spatial field h(r) = grad * (r . u) * e, sampled at the
    positions: strength linear in the coordinate along u = (cos, sin)(axis)
    (measured from the centre of the positions), direction e at angle_deg."""
    u = np.array([math.cos(math.radians(axis_deg)), math.sin(math.radians(axis_deg))])
    xy = np.asarray(xy, dtype=np.float64)
    r = (xy - xy.mean(axis=0)) @ u
    return _along(grad * r, angle_deg)


def travelling_wave(xy: np.ndarray, n_steps: int, amp: float, wavelength: float,
                    steps_per_period: int, angle_deg: float):
    """Spatial field of every step, h(r, t) = amp * sin(2 pi (x / wavelength
    - t / steps_per_period)) * e: a wave moving along x, direction e at
    angle_deg.  Returns [n_steps, n, 2]."""
    x = np.asarray(xy, dtype=np.float64)[:, 0]
    t = np.arange(int(n_steps), dtype=np.float64)[:, None]
    h = amp * np.sin(2.0 * np.pi * (x[None, :] / wavelength - t / float(steps_per_period)))
    a = math.radians(angle_deg)
    return np.ascontiguousarray(np.stack([h * math.cos(a), h * math.sin(a)], axis=2))


def random_local(n: int, n_slabs: int, amp: float, seed: int):
    """Independent N(0, amp^2) components per magnet (and per step when
    n_slabs > 1), numpy PCG64 from `seed`: [n, 2] or [n_slabs, n, 2]."""
    z = np.random.default_rng(int(seed)).standard_normal((int(n_slabs), int(n), 2)) * amp
    return np.ascontiguousarray(z[0] if n_slabs == 1 else z)


def exponential_anneal(n_steps: int, sigma0: float, sigma1: float):
    """Thermal std falling exponentially from sigma0 at the first step to
    sigma1 at the last (Sec. IV.B): sigma0 * (sigma1/sigma0)^(t/(K-1))."""
    K = int(n_steps)
    t = np.arange(K, dtype=np.float64) / max(1, K - 1)
    return np.ascontiguousarray(sigma0 * (sigma1 / sigma0) ** t)


# --------------------------------------------------------------------------
# random inputs
# --------------------------------------------------------------------------

def disorder_hk(n: int, hk_mean: float, k_disorder: float, seed: int) -> np.ndarray:
    """Per-magnet coercive fields h_k^(i) ~ N(h_k, k*h_k), kept positive
    (Sec. II.G); drawn with numpy's PCG64 generator from `seed`."""
    z = np.random.default_rng(int(seed)).standard_normal(int(n))
    hk = hk_mean + (k_disorder * hk_mean) * z
    return np.ascontiguousarray(np.maximum(hk, 1e-12 * hk_mean))


def polarised_spins(theta: np.ndarray, h0) -> np.ndarray:
    """Start spins along the first applied field: +1 where the island's
    axis has a non-negative projection on H[0], else -1."""
    h0 = np.asarray(h0, dtype=np.float64)
    nrm = float(np.hypot(h0[0], h0[1]))
    if nrm == 0.0:
        return np.ones(len(theta), dtype=np.int8)
    proj = np.cos(theta) * (h0[0] / nrm) + np.sin(theta) * (h0[1] / nrm)
    return np.where(proj >= 0.0, 1, -1).astype(np.int8)


# --------------------------------------------------------------------------
# workload bundles
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """Everything one simulation instance needs, as plain arrays + scalars."""
    name: str
    xy: np.ndarray          # [n,2] float64, lattice units
    theta: np.ndarray       # [n] float64, radians
    spin0: np.ndarray       # [n] int8, +-1
    hk: np.ndarray          # [n] float64 > 0
    H: np.ndarray           # [K,2] float64 applied field per step
    alpha: float
    neighbor_distance: float
    b: float
    c: float
    beta: float
    gamma: float
    thermal_std: float = 0.0
    thermal_seed: int = 0
    meta: Dict = dataclasses.field(default_factory=dict)
    # per-magnet external field added to H (Sec. II.D): [n,2] static or
    # [K,n,2] one slab per step; None for the global field alone
    h_loc: Optional[np.ndarray] = None
    # thermal std of each step (annealing, Sec. IV.B), replacing thermal_std
    sigma_t: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_steps(self) -> int:
        return int(self.H.shape[0])

    def params(self) -> Dict:
        return dict(alpha=self.alpha, neighbor_distance=self.neighbor_distance,
                    b=self.b, c=self.c, beta=self.beta, gamma=self.gamma,
                    thermal_std=self.thermal_std, thermal_seed=self.thermal_seed)

    def truncated(self, n_steps: int) -> "Workload":
        w = dataclasses.replace(self)
        w.H = np.ascontiguousarray(self.H[:int(n_steps)])
        return w


# Physics presets per geometry family (used by the named workloads and by the
# batched / served job generators).
SQUARE_PHYS = dict(alpha=0.001, b=1.0, c=1.0, beta=3.0, gamma=3.0, hk=0.2)
PINWHEEL_PHYS = dict(alpha=0.0013, b=0.38, c=1.0, beta=1.5, gamma=3.9, hk=0.2)
KAGOME_PHYS = dict(alpha=0.002, b=1.0, c=1.0, beta=3.0, gamma=3.0, hk=0.15)
FAMILY_PHYS = {"square": SQUARE_PHYS, "pinwheel": PINWHEEL_PHYS,
               "kagome": KAGOME_PHYS}


def square_10x10_triangle() -> Workload:
    """220-magnet square ASI, d=1, SW astroid, 200-step triangle at 45 deg."""
    xy, theta = square_closed(10)
    H = triangle_ramp(100, 0.3, 45.0)
    return Workload("square10_triangle", xy, theta,
                    np.ones(len(theta), dtype=np.int8),
                    disorder_hk(len(theta), 0.2, 0.05, 0), H,
                    alpha=0.001, neighbor_distance=1.0, b=1.0, c=1.0,
                    beta=3.0, gamma=3.0)


def pinwheel_100x100_reversal(n_steps: int = 2000) -> Workload:
    """20,200-magnet pinwheel, d=10, asymmetric astroid, reversal at 30 deg."""
    xy, theta = pinwheel_diamond(100)
    H = linear_ramp(2000, 0.1, -0.1, 30.0)[:n_steps]
    return Workload("pinwheel100_reversal", xy, theta,
                    polarised_spins(theta, H[0]),
                    disorder_hk(len(theta), 0.2, 0.05, 1), np.ascontiguousarray(H),
                    alpha=0.0013, neighbor_distance=10.0, b=0.38, c=1.0,
                    beta=1.5, gamma=3.9)


def pinwheel_300x300_reversal(n_steps: int = 2000) -> Workload:
    """180,600-magnet pinwheel at d = 10 (the 100 x 100 reversal's physics on
    a 300 x 300 array): ~105 M neighbour pairs, 2.1 GB of tables per
    full-field pass, far past the 256 MB last-level cache."""
    xy, theta = pinwheel_diamond(300)
    H = linear_ramp(2000, 0.1, -0.1, 30.0)[:n_steps]
    return Workload("pinwheel300_reversal", xy, theta,
                    polarised_spins(theta, H[0]),
                    disorder_hk(len(theta), 0.2, 0.05, 1), np.ascontiguousarray(H),
                    alpha=0.0013, neighbor_distance=10.0, b=0.38, c=1.0,
                    beta=1.5, gamma=3.9)


def kagome_1m_rotating(n_steps: int = 2000, cells: int = 577) -> Workload:
    """~1.0M-magnet kagome (577x577 cells), d=3, thermal std 0.005,
    rotating field of 0.08 with 1000 steps per revolution."""
    xy, theta = kagome(cells)
    H = rotating(2000, 0.08, 1000)[:n_steps]
    return Workload("kagome577_rotating", xy, theta,
                    polarised_spins(theta, H[0]),
                    disorder_hk(len(theta), 0.15, 0.05, 2), np.ascontiguousarray(H),
                    alpha=0.002, neighbor_distance=3.0, b=1.0, c=1.0,
                    beta=3.0, gamma=3.0, thermal_std=0.005, thermal_seed=2)


def square_anneal(side: int = 50, n_steps: int = 200, alpha: float = 0.0015) -> Workload:
    """Thermal annealing of closed-edge square ASI (Sec. IV.B): b = 0.4,
    c = 1, beta = gamma = 3, h_k ~ N(0.186, 0.05 * 0.186), neighbourhood 10,
    no applied field, thermal std falling exponentially 0.12 -> 0.004 over
    n_steps; all spins +1 at the start."""
    xy, theta = square_closed(side)
    n = len(theta)
    return Workload(f"square{side}_anneal", xy, theta, np.ones(n, np.int8),
                    disorder_hk(n, 0.186, 0.05, 3), np.zeros((int(n_steps), 2)),
                    alpha=alpha, neighbor_distance=10.0, b=0.4, c=1.0, beta=3.0, gamma=3.0,
                    thermal_std=0.0, thermal_seed=12,
                    sigma_t=exponential_anneal(n_steps, 0.12, 0.004))


NAMED = {
    "square10_triangle": square_10x10_triangle,
    "pinwheel100_reversal": pinwheel_100x100_reversal,
    "pinwheel300_reversal": pinwheel_300x300_reversal,
    "kagome577_rotating": kagome_1m_rotating,
    "square50_anneal": square_anneal,
}


def family_instance(family: str, n_target: int, d: float, seed: int,
                    H: np.ndarray, thermal_std: float = 0.0,
                    thermal_seed: int = 0, name: str = "") -> Workload:
    """One instance of a geometry family sized near n_target magnets."""
    phys = FAMILY_PHYS[family]
    if family == "kagome":
        xy, theta = kagome(kagome_cells_for(n_target))
    else:
        xy, theta = GEOMETRIES[family](square_side_for(n_target))
    return Workload(name or f"{family}{len(theta)}", xy, theta,
                    polarised_spins(theta, H[0]),
                    disorder_hk(len(theta), phys["hk"], 0.05, seed),
                    np.ascontiguousarray(H), alpha=phys["alpha"],
                    neighbor_distance=float(d), b=phys["b"], c=phys["c"],
                    beta=phys["beta"], gamma=phys["gamma"],
                    thermal_std=float(thermal_std), thermal_seed=int(thermal_seed))


def batched_sweep(count: int = 256, seed: int = 4, n_steps: int = 500,
                  side_range=(20, 200), distances=(1.0, 3.0, 10.0)) -> List[Workload]:
    """Uneven sweep of square / pinwheel instances, one linear ramp each.

    Family uniform over {square, pinwheel}; side U{lo..hi}; neighbour
    distance uniform over `distances`; disorder seeds 100, 101, ...; ramp
    +A -> -A at an angle U(0, 90) deg (A = 0.3 square, 0.1 pinwheel)."""
    rng = np.random.default_rng(int(seed))
    out = []
    for k in range(int(count)):
        fam = "square" if rng.integers(0, 2) == 0 else "pinwheel"
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        d = float(distances[int(rng.integers(0, len(distances)))])
        ang = float(rng.uniform(0.0, 90.0))
        amp = 0.3 if fam == "square" else 0.1
        H = linear_ramp(n_steps, amp, -amp, ang)
        xy, theta = GEOMETRIES[fam](side)
        phys = FAMILY_PHYS[fam]
        out.append(Workload(f"{fam}{side}_d{d:g}_{k}", xy, theta,
                            polarised_spins(theta, H[0]),
                            disorder_hk(len(theta), phys["hk"], 0.05, 100 + k), H,
                            alpha=phys["alpha"], neighbor_distance=d,
                            b=phys["b"], c=phys["c"], beta=phys["beta"],
                            gamma=phys["gamma"],
                            meta=dict(family=fam, side=side, angle=ang)))
    return out


@dataclasses.dataclass
class JobSpec:
    """A served simulation request (materialised lazily: arrays can be big)."""
    job: int
    arrival_s: float
    family: str
    n_target: int
    d: float
    protocol: str
    n_steps: int
    angle_deg: float
    thermal_std: float
    seed: int

    def workload(self) -> Workload:
        phys = FAMILY_PHYS[self.family]
        amp = {"square": 0.3, "pinwheel": 0.1, "kagome": 0.08}[self.family]
        if self.protocol == "ramp":
            H = linear_ramp(self.n_steps, amp, -amp, self.angle_deg)
        else:
            H = rotating(self.n_steps, amp, max(2, self.n_steps // 2), self.angle_deg)
        del phys
        return family_instance(self.family, self.n_target, self.d, self.seed, H,
                               self.thermal_std, self.seed,
                               name=f"job{self.job}_{self.family}")


def served_stream(count: int = 2000, seed: int = 5, rate_per_s: float = 50.0,
                  n_range=(1e3, 1e6), steps_range=(100, 2000)) -> List[JobSpec]:
    """Poisson arrival stream of mixed-size simulation requests."""
    rng = np.random.default_rng(int(seed))
    t = 0.0
    jobs = []
    for k in range(int(count)):
        t += float(rng.exponential(1.0 / rate_per_s))
        fam = ("square", "pinwheel", "kagome")[int(rng.integers(0, 3))]
        n_t = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        d = float(rng.integers(1, 11))
        proto = "ramp" if rng.integers(0, 2) == 0 else "rotating"
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        ang = float(rng.uniform(0.0, 90.0))
        th = 0.0 if rng.integers(0, 2) == 0 else float(rng.uniform(0.0, 0.01))
        jobs.append(JobSpec(k, t, fam, n_t, d, proto, steps, ang, th, 1000 + k))
    return jobs


def random_cloud(n: int, seed: int, box: float = None, min_sep: float = 0.3):
    """Random positions (rejection-sampled to keep a minimum separation) and
    random angles, for brute-force and property tests on arbitrary 2-D
    geometries (Sec. II.I: any 2-D arrangement of identical islands)."""
    rng = np.random.default_rng(int(seed))
    box = box if box is not None else math.sqrt(n) * 1.2
    pts = []
    tries = 0
    while len(pts) < n:
        p = rng.uniform(0.0, box, size=2)
        tries += 1
        if all((p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2 >= min_sep ** 2 for q in pts):
            pts.append(p)
        if tries > 200 * n:
            raise RuntimeError("random_cloud: box too small for min_sep")
    xy = np.ascontiguousarray(np.array(pts, dtype=np.float64))
    theta = np.ascontiguousarray(rng.uniform(0.0, np.pi, size=n))
    return xy, theta
