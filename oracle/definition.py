"""Oracle, tier 0: the flatspin dipole model written out literally in numpy.

TEST INFRASTRUCTURE ONLY: the product path never imports this module; only
tests/, the package smoke check and the benchmark's CPU-baseline leg do.

Every function follows one passage of the paper (Jensen et al., flatspin,
Sec. II) with no blocking, caching or incremental update: after every single
flip, *all* fields are recomputed from Eq. 3, exactly as Sec. II.H describes.
It is meant for tiny inputs (a few hundred magnets).
"""
from __future__ import annotations

import numpy as np

CUTOFF_SLACK = 1e-9

# Philox4x32-10 constants (Salmon et al., SC'11: round multipliers and the
# two Weyl key increments).
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def unit_vectors(theta):
    """Eq. 1: mhat_i = (cos th_i, sin th_i); the perpendicular (hard) axis
    mhat_perp_i = (-sin th_i, cos th_i) (Sec. II.F, Fig. 2a)."""
    m = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    p = np.stack([-m[:, 1], m[:, 0]], axis=1)
    return m, p


def neighbour_mask(xy, d):
    """Sec. II.C: neighbourhood = magnets j != i within distance d (lattice
    units), inclusive.  Brute force over all pairs."""
    dx = xy[:, None, 0] - xy[None, :, 0]
    dy = xy[:, None, 1] - xy[None, :, 1]
    cut = d + CUTOFF_SLACK
    mask = dx * dx + dy * dy <= cut * cut
    np.fill_diagonal(mask, False)
    return mask


def dipolar_field(xy, theta, spins, alpha, mask):
    """Eq. 3: h_dip_i = alpha * sum_{j in N(i)} 3 r (m_j.r)/|r|^5 - m_j/|r|^3,
    with r = r_i - r_j and m_j = s_j mhat_j (Eq. 1).  Returns [n, 2]."""
    m, _ = unit_vectors(theta)
    mj = spins[:, None].astype(np.float64) * m
    n = len(xy)
    h = np.zeros((n, 2))
    for i in range(n):
        js = np.nonzero(mask[i])[0]
        if len(js) == 0:
            continue
        r = xy[i][None, :] - xy[js]
        rn = np.sqrt(np.sum(r * r, axis=1))
        mr = np.sum(mj[js] * r, axis=1)
        term = 3.0 * r * (mr / rn ** 5)[:, None] - mj[js] / (rn ** 3)[:, None]
        h[i] = alpha * term.sum(axis=0)
    return h


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds over arrays: ctr [..., 4], key [..., 2]
    (uint32 values held in uint64).  Returns [..., 4]."""
    c = [np.asarray(ctr[..., k], dtype=np.uint64) for k in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(_W0)) & np.uint64(_MASK)
            k1 = (k1 + np.uint64(_W1)) & np.uint64(_MASK)
        p0 = np.uint64(_M0) * c[0]
        p1 = np.uint64(_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def normal_pairs(seed, c0, c1, tag=0):
    """Two N(0,1) draws per counter (c0, c1, tag, 0) by Box-Muller over the
    Philox output: u1 = (top 53 bits of words 0,1 + 1) * 2^-53 in (0, 1],
    u2 = (top 53 bits of words 2,3) * 2^-53 in [0, 1)."""
    c0 = np.atleast_1d(np.asarray(c0, dtype=np.uint64))
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), c0.shape)
    ctr = np.stack([c0, c1, np.full_like(c0, tag), np.zeros_like(c0)], axis=-1)
    seed = int(seed)
    key = np.broadcast_to(np.array([seed & _MASK, (seed >> 32) & _MASK],
                                   dtype=np.uint64), c0.shape + (2,))
    o = philox4x32_10(ctr, key)
    a = ((o[..., 0] << np.uint64(32)) | o[..., 1]) >> np.uint64(11)
    b = ((o[..., 2] << np.uint64(32)) | o[..., 3]) >> np.uint64(11)
    u1 = (a + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 6.283185307179586 * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def thermal_field(n, t, sigma, seed):
    """Sec. II.E: per magnet, two orthogonal components ~ N(0, sigma^2),
    drawn once per field step t (counter (i, t, 0, 0)).  Returns [n, 2]."""
    if sigma == 0.0:
        return np.zeros((n, 2))
    z0, z1 = normal_pairs(seed, np.arange(n, dtype=np.uint64), np.uint64(t), 0)
    return np.stack([sigma * z0, sigma * z1], axis=1)


def projections(h, theta):
    """h_par = h.mhat, h_perp = h.mhat_perp (Sec. II.F)."""
    m, p = unit_vectors(theta)
    return np.sum(h * m, axis=1), np.sum(h * p, axis=1)


def astroid_lhs(h_par, h_perp, hk, b, c, beta, gamma):
    """Left-hand side of the generalized Stoner-Wohlfarth astroid, Eq. 5,
    on |h_par|, |h_perp|."""
    return (np.abs(h_par) / (b * hk)) ** (2.0 / gamma) + \
        (np.abs(h_perp) / (c * hk)) ** (2.0 / beta)


def flippable(spins, h_par, lhs):
    """Eq. 5 > 1 (strict) and Eq. 6: h . m < 0, i.e. s_i h_par_i < 0."""
    return (spins * h_par < 0.0) & (lhs > 1.0)


class Model:
    """One instance: geometry, astroid, disorder, temperature (Sec. II)."""

    def __init__(self, xy, theta, hk, alpha, neighbor_distance, b, c, beta,
                 gamma, thermal_std=0.0, thermal_seed=0, **_):
        self.xy = np.asarray(xy, dtype=np.float64)
        self.theta = np.asarray(theta, dtype=np.float64)
        self.hk = np.asarray(hk, dtype=np.float64)
        self.alpha = float(alpha)
        self.b, self.c, self.beta, self.gamma = map(float, (b, c, beta, gamma))
        self.sigma = float(thermal_std)
        self.seed = int(thermal_seed)
        self.mask = neighbour_mask(self.xy, float(neighbor_distance))

    @property
    def n(self):
        return len(self.xy)

    def total_field(self, spins, H, t):
        """Eq. 2: h_i = h_dip + h_ext + h_th, then projected."""
        h = dipolar_field(self.xy, self.theta, spins, self.alpha, self.mask)
        h = h + np.asarray(H, dtype=np.float64)[None, :]
        h = h + thermal_field(self.n, t, self.sigma, self.seed)
        return projections(h, self.theta)

    def relax(self, spins, H, t, log):
        """Sec. II.H: flip the flippable magnet with the greatest Eq. 5 LHS
        (ties: lowest index), recompute every field, repeat until stable."""
        while True:
            hp, hq = self.total_field(spins, H, t)
            lhs = astroid_lhs(hp, hq, self.hk, self.b, self.c, self.beta, self.gamma)
            ok = flippable(spins, hp, lhs)
            if not ok.any():
                return hp, hq
            j = int(np.argmax(np.where(ok, lhs, -np.inf)))  # first max = lowest i
            spins[j] = -spins[j]
            log.append((t, j))

    def run(self, spins, Hs, t_begin=0, t_end=None):
        """Field steps t_begin..t_end-1: set H[t] and h_th(t), relax."""
        spins = np.array(spins, dtype=np.int8)
        t_end = len(Hs) if t_end is None else t_end
        log = []
        hp = hq = None
        for t in range(t_begin, t_end):
            hp, hq = self.relax(spins, Hs[t], t, log)
        return spins, log, hp, hq
