"""ctypes binding of the tier-1 C++ oracle (relax.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "relax.cpp")
LIB = os.path.join(HERE, "liborc.so")

_lib = None
# FNV-1a 64-bit offset basis: the checksum of an empty flip log
FNV_OFFSET = 14695981039346656037


def build(force: bool = True) -> str:
    """Compile relax.cpp with g++ (FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-std=c++17",
                               "-fPIC", "-shared", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.c_int64, dp, dp, dp] + [C.c_double] * 7 + [C.c_uint64]
        L.orc_destroy.argtypes = [P]
        L.orc_num_edges.restype = C.c_int64
        L.orc_num_edges.argtypes = [P]
        L.orc_neighbours.argtypes = [P, C.c_void_p, C.c_void_p]
        L.orc_set_spins.argtypes = [P, C.c_void_p]
        L.orc_get_spins.argtypes = [P, C.c_void_p]
        L.orc_set_local_field.argtypes = [P, C.c_int64, C.c_void_p]
        L.orc_set_thermal_schedule.argtypes = [P, C.c_int64, C.c_void_p]
        L.orc_fields.argtypes = [P, dp, C.c_int64] + [C.c_void_p] * 5
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [P, C.c_int64, dp, C.c_int64, C.c_int64, C.c_void_p,
                              C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_void_p,
                              C.c_void_p, C.c_int64, C.POINTER(C.c_uint64), C.c_void_p]
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_normal_pair.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_void_p]
        L.orc_disorder_hk.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_uint64, C.c_void_p]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vp(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_vp(c), _vp(k), _vp(o))
    return o


def normal_pair(seed, c0, c1, tag=0):
    z = np.zeros(2)
    lib().orc_normal_pair(int(seed), int(c0), int(c1), int(tag), _vp(z))
    return z


def disorder_hk(n, mean, k, seed):
    """Coercive fields drawn from the disorder distribution (Sec. II.G):
    mean + (k * mean) * z_i, z_i the first normal of counter (i, 0, 1, 0),
    raised to 1e-12 * mean where below."""
    out = np.zeros(int(n))
    lib().orc_disorder_hk(int(n), float(mean), float(k), int(seed), _vp(out))
    return out


class Oracle:
    """One model instance held by the C++ oracle."""

    def __init__(self, xy, theta, hk, alpha, neighbor_distance, b, c, beta, gamma,
                 thermal_std=0.0, thermal_seed=0, **_):
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.hk = np.ascontiguousarray(hk, dtype=np.float64)
        self.n = len(self.theta)
        self.alpha = float(alpha)
        self._h = lib().orc_create(self.n, _dp(self.xy), _dp(self.theta), _dp(self.hk),
                                   alpha, neighbor_distance, b, c, beta, gamma,
                                   thermal_std, int(thermal_seed))
        if not self._h:
            raise ValueError("oracle: bad instance")

    @classmethod
    def from_workload(cls, w):
        o = cls(w.xy, w.theta, w.hk, **w.params())
        if getattr(w, "h_loc", None) is not None:
            o.set_local_field(w.h_loc)
        if getattr(w, "sigma_t", None) is not None:
            o.set_thermal_schedule(w.sigma_t)
        return o

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_edges(self):
        return int(lib().orc_num_edges(self._h))

    def neighbours(self):
        ptr = np.zeros(self.n + 1, dtype=np.int64)
        idx = np.zeros(max(1, self.num_edges), dtype=np.int32)
        lib().orc_neighbours(self._h, _vp(ptr), _vp(idx))
        return ptr, idx[:self.num_edges]

    def set_spins(self, s):
        s = np.ascontiguousarray(s, dtype=np.int8)
        lib().orc_set_spins(self._h, _vp(s))

    def spins(self):
        s = np.zeros(self.n, dtype=np.int8)
        lib().orc_get_spins(self._h, _vp(s))
        return s

    def set_local_field(self, h_loc):
        """Local external field (Sec. II.D): (n, 2) for every step, (K, n, 2)
        one slab per step, None for none.  Adds to any wave set below."""
        self._user_loc = None if h_loc is None else np.ascontiguousarray(h_loc, dtype=np.float64)
        if self._user_loc is not None and self._user_loc.ndim == 2:
            self._user_loc = self._user_loc[None]
        if self._user_loc is not None:
            assert self._user_loc.ndim == 3 and self._user_loc.shape[1:] == (self.n, 2)
        self._push_local()

    def set_local_wave(self, amp, kx, ky, period_steps, phase0, angle_rad, n_steps):
        """Travelling-wave local field of each step t < n_steps:
        amp sin(2 pi (kx x_i + ky y_i) + phase0 - 2 pi t / period_steps)
        along (cos, sin)(angle); amp = 0 removes it."""
        if amp == 0.0:
            self._wave = None
        else:
            t = np.arange(int(n_steps), dtype=np.float64)[:, None]
            arg = 2.0 * np.pi * (kx * self.xy[:, 0] + ky * self.xy[:, 1])[None, :] + phase0 \
                - 2.0 * np.pi * t / period_steps
            a = amp * np.sin(arg)
            self._wave = np.stack([a * math.cos(angle_rad), a * math.sin(angle_rad)], axis=2)
        self._push_local()

    def _push_local(self):
        loc = getattr(self, "_user_loc", None)
        wave = getattr(self, "_wave", None)
        if loc is None and wave is None:
            self._loc, self._loc_k = None, 0
            lib().orc_set_local_field(self._h, 0, None)
            return
        if wave is None:
            a = loc
        elif loc is None:
            a = wave
        else:
            a = wave + loc      # a static field broadcasts over the wave's steps
        a = np.ascontiguousarray(a)
        self._loc, self._loc_k = a, a.shape[0]
        lib().orc_set_local_field(self._h, a.shape[0], _vp(a))

    def set_thermal_schedule(self, sigma):
        """Thermal std per step (annealing, Sec. IV.B), or None."""
        a = np.zeros(0) if sigma is None else np.ascontiguousarray(sigma, dtype=np.float64)
        self._sig = a
        lib().orc_set_thermal_schedule(self._h, len(a), _vp(a) if len(a) else None)

    def magnetization(self, spins=None):
        """Net magnetisation sum_i s_i mhat_i (Eq. 1 summed over the array),
        for the current spins or the given ones."""
        s = (self.spins() if spins is None else np.asarray(spins)).astype(np.float64)
        return np.array([np.sum(s * np.cos(self.theta)), np.sum(s * np.sin(self.theta))])

    def group_magnetization(self, ptr, idx, spins=None):
        """[G, 2]: sum of s_i mhat_i over each CSR group (a vertex map when
        the groups are the islands meeting at each vertex)."""
        s = (self.spins() if spins is None else np.asarray(spins)).astype(np.float64)
        out = np.zeros((len(ptr) - 1, 2))
        for g in range(len(ptr) - 1):
            for i in idx[ptr[g]:ptr[g + 1]]:
                out[g, 0] += s[i] * math.cos(self.theta[i])
                out[g, 1] += s[i] * math.sin(self.theta[i])
        return out

    def spin_correlation(self, bin_width, n_bins, spins=None):
        """(sums, counts) per distance bin of the pair correlation (Sec.
        IV.B): +1 when the pair's dipolar energy -s_i s_j A_ij is minimal,
        -1 when maximal, 0 when A_ij vanishes (|A_ij| <= 1e-9 |alpha| / r^3),
        A_ij = alpha mhat_i . (3 r (mhat_j . r) / |r|^5 - mhat_j / |r|^3)
        from Eq. 3 with r = r_i - r_j; each neighbour pair once, in bin
        floor(r / w)."""
        s = self.spins() if spins is None else np.asarray(spins, dtype=np.int64)
        ptr, idx = self.neighbours()
        sums = np.zeros(int(n_bins), dtype=np.int64)
        cnts = np.zeros(int(n_bins), dtype=np.int64)
        m = np.stack([np.cos(self.theta), np.sin(self.theta)], 1)
        for i in range(self.n):
            js = idx[ptr[i]:ptr[i + 1]]
            js = js[js > i]
            if len(js) == 0:
                continue
            d = self.xy[i] - self.xy[js]
            r = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1])
            b = np.floor(r / bin_width)
            mj = m[js]
            proj = (mj * d).sum(1)
            g = 3.0 * d * (proj / r ** 5)[:, None] - mj / (r ** 3)[:, None]
            A = self.alpha * (g @ m[i])
            c = np.where(np.abs(A) > 1e-9 * abs(self.alpha) / r ** 3,
                         np.where(int(s[i]) * s[js] * np.sign(A) > 0, 1, -1), 0)
            ok = b < n_bins
            np.add.at(sums, b[ok].astype(np.int64), c[ok])
            np.add.at(cnts, b[ok].astype(np.int64), 1)
        return sums, cnts

    def fields(self, H, t):
        """(h_par, h_perp, scale) for the current spins at step t."""
        assert getattr(self, "_loc_k", 0) <= 1 or t < self._loc_k
        assert len(getattr(self, "_sig", ())) == 0 or t < len(self._sig)
        H = np.ascontiguousarray(H, dtype=np.float64)
        hp, hq, sc = (np.zeros(self.n) for _ in range(3))
        lib().orc_fields(self._h, _dp(H), int(t), _vp(hp), _vp(hq), None, None, _vp(sc))
        return hp, hq, sc

    def dipolar_xy(self):
        hx, hy = np.zeros(self.n), np.zeros(self.n)
        H = np.zeros(2)
        lib().orc_fields(self._h, _dp(H), 0, None, None, _vp(hx), _vp(hy), None)
        return hx, hy

    def run(self, Hs, t_begin=0, t_end=None, log_cap=None, max_flips_per_step=0,
            fnv=FNV_OFFSET):
        """Run steps; returns dict(status, flips (t, j) arrays, per_step, gaps,
        hash, step_top2).  `hash` is the FNV-1a checksum of every flip of the
        call (stored in the log or not), continued from `fnv`; `step_top2`
        the smallest top-two relative key gap of each step."""
        Hs = np.ascontiguousarray(Hs, dtype=np.float64)
        K = len(Hs)
        t_end = K if t_end is None else int(t_end)
        cap = int(log_cap) if log_cap is not None else 4 * self.n * max(1, t_end - t_begin) // 10 + 1024
        cap = max(cap, 1024)
        lt = np.zeros(cap, dtype=np.int32)
        lj = np.zeros(cap, dtype=np.int32)
        per = np.zeros(max(1, t_end - t_begin), dtype=np.int32)
        top2 = np.zeros(max(1, t_end - t_begin))
        gaps = np.zeros(3)
        nf = C.c_int64(0)
        h = C.c_uint64(int(fnv))
        st = lib().orc_run(self._h, K, _dp(Hs), int(t_begin), t_end, _vp(lt), _vp(lj),
                           cap, C.byref(nf), _vp(per), _vp(gaps), int(max_flips_per_step),
                           C.byref(h), _vp(top2))
        n = nf.value
        return dict(status=int(st), n_flips=n, step=lt[:min(n, cap)].copy(),
                    idx=lj[:min(n, cap)].copy(), truncated=n > cap,
                    per_step=per[:t_end - t_begin].copy(), hash=h.value,
                    step_top2=top2[:t_end - t_begin].copy(),
                    gaps=dict(top2_rel=gaps[0], thresh_rel=gaps[1], par_rel=gaps[2]))
