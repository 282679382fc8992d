"""Python binding of the C ABI in include/asi.h (argument marshalling only).

Every step of the model runs in the HIP kernels of libasi.so; this module
only converts numpy arrays to pointers and status codes to exceptions.
PyTorch, when used, supplies the HIP stream and the caching allocator for
the library's device memory.  There is no CPU fallback: without the built
library, or without a GPU, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ASI_LIBRARY may point at another build of the same library (kernel variants)
LIB_PATH = os.environ.get("ASI_LIBRARY") or os.path.join(HERE, "libasi.so")

ASI_OK, ASI_EINVAL, ASI_ENOMEM, ASI_EDEVICE, ASI_ESTATE, ASI_ELOOP, ASI_EBUSY = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "ASI_OK", -1: "ASI_EINVAL", -2: "ASI_ENOMEM", -3: "ASI_EDEVICE",
                -4: "ASI_ESTATE", -5: "ASI_ELOOP", -6: "ASI_EBUSY"}
# asi_params.field_mode: carry the dipolar sums across steps by the flip
# deltas, re-gather rows whose neighbours flipped, or re-gather every row
FIELD_MODES = {"carry": 0, "dirty": 1, "full": 2}
# Astroid parameters that reduce Eq. 5 to the parallel-only switching test
# -s_i h_par > h_k^(i) (Sec. IV.C): no hard-axis term, exponent 1.
PARALLEL_CRITERION = dict(b=1.0, c=float("inf"), gamma=2.0)
# asi_batch_run modes
BATCH_MODES = {"lockstep": 0, "graph": 1, "fused": 2}
FNV_OFFSET = 0xcbf29ce484222325
FNV_PRIME = 0x100000001b3

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class AsiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class AsiDevice(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("ctx", C.c_void_p)]


class AsiParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n", C.c_int64), ("xy", C.c_void_p),
                ("theta", C.c_void_p), ("spin0", C.c_void_p), ("hk", C.c_void_p),
                ("alpha", C.c_double), ("neighbor_distance", C.c_double),
                ("b", C.c_double), ("c", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("thermal_std", C.c_double),
                ("thermal_seed", C.c_uint64), ("max_flips_per_step", C.c_int64),
                ("flip_log_capacity", C.c_int64), ("field_mode", C.c_int32),
                ("hk_mean", C.c_double), ("k_disorder", C.c_double),
                ("disorder_seed", C.c_uint64)]


class AsiInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_edges", C.c_int64), ("max_degree", C.c_int32),
                ("relax_waves", C.c_int32), ("device_bytes", C.c_int64),
                ("field_pass_bytes", C.c_double), ("flip_log_capacity", C.c_int64)]


class AsiTiming(C.Structure):
    _fields_ = [("field_launches", C.c_int64), ("field_ms", C.c_double),
                ("relax_launches", C.c_int64), ("relax_ms", C.c_double)]


class AsiTuning(C.Structure):
    _fields_ = [("relax_waves", C.c_int32), ("l1_shift", C.c_int32), ("spec_min", C.c_int64),
                ("default_ms", C.c_double), ("tuned_ms", C.c_double), ("trials", C.c_int32),
                ("field_rows", C.c_int32)]


class AsiServerStats(C.Structure):
    _fields_ = [("bursts", C.c_int64), ("admitted", C.c_int64), ("retired", C.c_int64),
                ("pauses", C.c_int64), ("admit_s", C.c_double), ("wait_s", C.c_double),
                ("retire_s", C.c_double), ("rebuild_s", C.c_double)]


# Every entry point of include/asi.h with its ctypes signature.
P = C.c_void_p
I64P = C.POINTER(C.c_int64)
SIGNATURES = {
    "asi_create": [C.POINTER(AsiParams), C.POINTER(AsiDevice), C.POINTER(C.c_void_p)],
    "asi_set_field_protocol": [P, C.c_int64, P],
    "asi_set_local_field": [P, C.c_int64, P],
    "asi_set_thermal_schedule": [P, C.c_int64, P],
    "asi_set_local_wave": [P, P] + [C.c_double] * 6,
    "asi_magnetization": [P, P],
    "asi_spin_correlation": [P, P, C.c_double, C.c_int32, P, P],
    "asi_group_magnetization": [P, C.c_int64, P, P, P],
    "asi_switching_order": [P, P],
    "asi_switching_rho": [P, P, C.POINTER(C.c_double), P],
    "asi_switching_rho_noalloc": [P, P, C.POINTER(C.c_double), P],
    "asi_set_magnetization_log": [P, C.c_int32],
    "asi_get_magnetization_log": [P, P],
    "asi_relax": [P, I64P],
    "asi_run": [P, C.c_int64, C.c_int64, I64P],
    "asi_get_state": [P, P, P, P, I64P],
    "asi_set_state": [P, P, C.c_int64],
    "asi_get_flip_log": [P, C.c_int64, P, P, I64P, C.POINTER(C.c_uint64)],
    "asi_get_step_flips": [P, P],
    "asi_compute_fields": [P, C.c_int64],
    "asi_get_info": [P, C.POINTER(AsiInfo)],
    "asi_set_timing": [P, C.c_int32],
    "asi_get_timing": [P, C.POINTER(AsiTiming)],
    "asi_destroy": [P],
    "asi_last_error": [],
    "asi_batch_run": [P, C.c_int32, C.c_int32, P],
    "asi_server_create": [C.POINTER(AsiDevice), C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)],
    "asi_server_submit": [P, C.POINTER(AsiParams), C.c_int64, P, I64P],
    "asi_server_submit_fields": [P, C.POINTER(AsiParams), C.c_int64, P, C.c_int64, P, P, I64P],
    "asi_server_step": [P, C.c_double, C.POINTER(C.c_int32)],
    "asi_server_poll": [P, C.c_int64, C.POINTER(C.c_int32)],
    "asi_server_take": [P, C.c_int64, P, I64P, C.POINTER(C.c_uint64),
                        C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "asi_server_get_stats": [P, C.POINTER(AsiServerStats)],
    "asi_tune": [P, C.c_int64, C.POINTER(AsiTuning)],
    "asi_get_tuning": [P, C.POINTER(AsiTuning)],
    "asi_set_tuning": [P, C.POINTER(AsiTuning)],
    "asi_server_destroy": [P],
    "asi_measure_load_latency": [C.POINTER(AsiDevice), C.c_int64, C.c_int64, C.c_int32,
                                 C.c_uint64, C.POINTER(C.c_double)],
}

_lib = None


def library():
    """Load libasi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2002_11401_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_char_p if name == "asi_last_error" else C.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != ASI_OK:
        raise AsiError(st, library().asi_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def flip_hash(steps, idx) -> int:
    """The flip-log hash defined in include/asi.h, for a (step, index) list."""
    h = FNV_OFFSET
    for t, j in zip(steps, idx):
        w = ((int(t) & 0xFFFFFFFF) << 32) | (int(j) & 0xFFFFFFFF)
        h = ((h ^ w) * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


class _TorchDevice:
    """asi_device backed by PyTorch's current stream and caching allocator."""

    def __init__(self):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch; the HIP library needs one")
        self.torch = torch
        self.dev = torch.cuda.current_device()
        self.stream = torch.cuda.current_stream()
        torch_ = torch
        dev = self.dev
        stream = self.stream

        def _alloc(nbytes, _st, _ctx):
            try:
                return torch_.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except Exception:
                return None

        def _free(p, _st, _ctx):
            if p:
                torch_.cuda.caching_allocator_delete(p)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = AsiDevice(C.c_void_p(self.stream.cuda_stream), self._alloc, self._free, None)


def make_device(kind: str = "torch"):
    """'torch': torch stream + caching allocator; 'hip': library-owned stream
    and hipMalloc."""
    if kind == "torch":
        return _TorchDevice()
    if kind == "hip":
        class _Plain:
            struct = AsiDevice(None, ALLOC_FN(), FREE_FN(), None)
        return _Plain()
    raise ValueError(kind)


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


def _params(xy, theta, hk, spin0, alpha, neighbor_distance, b, c, beta, gamma,
            thermal_std=0.0, thermal_seed=0, max_flips_per_step=0, flip_log_capacity=0,
            field_mode="carry", hk_mean=0.0, k_disorder=0.0, disorder_seed=0):
    """hk None: the library draws the coercive fields from hk_mean,
    k_disorder and disorder_seed (see asi_params in include/asi.h)."""
    keep = [np.ascontiguousarray(xy, dtype=np.float64).reshape(-1),
            np.ascontiguousarray(theta, dtype=np.float64),
            None if hk is None else np.ascontiguousarray(hk, dtype=np.float64),
            None if spin0 is None else np.ascontiguousarray(spin0, dtype=np.int8)]
    n = len(keep[1])
    if (len(keep[0]) != 2 * n or (keep[2] is not None and len(keep[2]) != n) or
            (keep[3] is not None and len(keep[3]) != n)):
        raise ValueError("xy must be [n,2]; theta, hk, spin0 must be [n]")
    p = AsiParams(C.sizeof(AsiParams), n, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[3]),
                  _ptr(keep[2]), float(alpha), float(neighbor_distance), float(b), float(c),
                  float(beta), float(gamma), float(thermal_std), int(thermal_seed),
                  int(max_flips_per_step), int(flip_log_capacity),
                  FIELD_MODES[field_mode] if isinstance(field_mode, str) else int(field_mode),
                  float(hk_mean), float(k_disorder), int(disorder_seed))
    return p, keep


class Sim:
    """One simulation instance held by the HIP library."""

    def __init__(self, xy, theta, hk, spin0=None, *, alpha, neighbor_distance, b, c, beta,
                 gamma, thermal_std=0.0, thermal_seed=0, H=None, max_flips_per_step=0,
                 flip_log_capacity=0, field_mode="carry", device="torch", hk_mean=0.0,
                 k_disorder=0.0, disorder_seed=0):
        L = library()
        self._dev = device if not isinstance(device, str) else make_device(device)
        p, keep = _params(xy, theta, hk, spin0, alpha, neighbor_distance, b, c, beta, gamma,
                          thermal_std, thermal_seed, max_flips_per_step, flip_log_capacity,
                          field_mode, hk_mean, k_disorder, disorder_seed)
        h = C.c_void_p()
        _check(L.asi_create(C.byref(p), C.byref(self._dev.struct), C.byref(h)))
        self._h = h
        self.n = len(keep[1])
        self.K = 0
        _live.add(self)
        if H is not None:
            self.set_protocol(H)

    @classmethod
    def from_workload(cls, w, device="torch", **kw):
        sim = cls(w.xy, w.theta, w.hk, w.spin0, H=w.H, device=device, **w.params(), **kw)
        if getattr(w, "h_loc", None) is not None:
            sim.set_local_field(w.h_loc)
        if getattr(w, "sigma_t", None) is not None:
            sim.set_thermal_schedule(w.sigma_t)
        return sim

    @property
    def handle(self):
        if not self._h:
            raise AsiError(ASI_ESTATE, "closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            library().asi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_protocol(self, H):
        H = np.ascontiguousarray(H, dtype=np.float64).reshape(-1, 2)
        _check(library().asi_set_field_protocol(self.handle, len(H), _ptr(H)))
        self.K = len(H)

    def set_local_field(self, h_loc):
        """Per-magnet external field added to H[t] (Sec. II.D): an (n, 2)
        array applies at every step, a (K, n, 2) array gives step t its own
        slab; None removes it."""
        if h_loc is None:
            _check(library().asi_set_local_field(self.handle, 0, None))
            return
        a = np.ascontiguousarray(h_loc, dtype=np.float64)
        if a.ndim == 2:
            a = a[None]
        if a.ndim != 3 or a.shape[1] != self.n or a.shape[2] != 2:
            raise ValueError("h_loc must be (n, 2) or (K, n, 2)")
        _check(library().asi_set_local_field(self.handle, a.shape[0], _ptr(a)))

    def set_local_wave(self, xy, amp, kx, ky, period_steps, phase0=0.0, angle_deg=0.0):
        """Travelling-wave local field evaluated on the device: amp * sin(2 pi
        (kx x + ky y) + phase0 - 2 pi t / period_steps) along angle_deg;
        amp = 0 removes it."""
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        if len(xy) != self.n:
            raise ValueError("xy must hold the n positions")
        _check(library().asi_set_local_wave(self.handle, _ptr(xy), float(amp), float(kx),
                                            float(ky), float(period_steps), float(phase0),
                                            np.deg2rad(float(angle_deg))))

    def set_thermal_schedule(self, sigma):
        """Thermal std of every step (length K), or None for thermal_std."""
        if sigma is None:
            _check(library().asi_set_thermal_schedule(self.handle, 0, None))
            return
        a = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1)
        if len(a) != self.K:
            raise ValueError("the schedule needs one value per protocol step")
        _check(library().asi_set_thermal_schedule(self.handle, len(a), _ptr(a)))

    def magnetization(self) -> np.ndarray:
        """Net magnetisation sum_i s_i mhat_i of the current spins, (x, y)."""
        m = np.zeros(2)
        _check(library().asi_magnetization(self.handle, _ptr(m)))
        return m

    def spin_correlation(self, xy, bin_width: float, n_bins: int):
        """(sums, counts) of the pair correlation per distance bin over the
        neighbour pairs; xy are the instance's positions."""
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        if len(xy) != self.n:
            raise ValueError("xy must hold the n positions")
        s = np.zeros(int(n_bins), dtype=np.int64)
        c = np.zeros(int(n_bins), dtype=np.int64)
        _check(library().asi_spin_correlation(self.handle, _ptr(xy), float(bin_width),
                                              int(n_bins), _ptr(s), _ptr(c)))
        return s, c

    def group_magnetization(self, ptr, idx) -> np.ndarray:
        """[G, 2]: net magnetisation of each CSR group of magnets (e.g. the
        islands of each vertex)."""
        ptr = np.ascontiguousarray(ptr, dtype=np.int64)
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        if len(ptr) < 2 or ptr[-1] > len(idx):
            raise ValueError("ptr must have G+1 entries ending at most at len(idx)")
        out = np.zeros((len(ptr) - 1, 2))
        idx_buf = idx if len(idx) else np.zeros(1, np.int32)   # held across the call
        _check(library().asi_group_magnetization(self.handle, len(ptr) - 1, _ptr(ptr),
                                                 _ptr(idx_buf), _ptr(out)))
        return out

    def switching_order(self) -> np.ndarray:
        """[n]: flip-log position of each magnet's first switch (the log's
        length for magnets that never switched), computed on the device."""
        out = np.zeros(self.n, dtype=np.int64)
        _check(library().asi_switching_order(self.handle, _ptr(out)))
        return out

    def set_magnetization_log(self, on: bool = True):
        _check(library().asi_set_magnetization_log(self.handle, 1 if on else 0))

    def magnetization_log(self) -> np.ndarray:
        """[K, 2]: M after the relax of each step run since the log was
        enabled (NaN for steps not run)."""
        out = np.zeros((max(1, self.K), 2))
        _check(library().asi_get_magnetization_log(self.handle, _ptr(out)))
        return out[:self.K]

    def run(self, t_begin=0, t_end=None) -> int:
        t_end = self.K if t_end is None else int(t_end)
        f = C.c_int64(0)
        _check(library().asi_run(self.handle, int(t_begin), t_end, C.byref(f)))
        return f.value

    def relax(self) -> int:
        f = C.c_int64(0)
        _check(library().asi_relax(self.handle, C.byref(f)))
        return f.value

    def compute_fields(self, t: int):
        _check(library().asi_compute_fields(self.handle, int(t)))

    def state(self):
        s = np.zeros(self.n, dtype=np.int8)
        hp = np.zeros(self.n)
        hq = np.zeros(self.n)
        step = C.c_int64(0)
        _check(library().asi_get_state(self.handle, _ptr(s), _ptr(hp), _ptr(hq), C.byref(step)))
        return s, hp, hq, step.value

    def set_state(self, spins, step: int):
        s = np.ascontiguousarray(spins, dtype=np.int8)
        if len(s) != self.n:
            raise ValueError("spins must have n entries")
        _check(library().asi_set_state(self.handle, _ptr(s), int(step)))

    def flip_log(self, cap: Optional[int] = None):
        cnt = C.c_int64(0)
        h = C.c_uint64(0)
        _check(library().asi_get_flip_log(self.handle, 0, None, None, C.byref(cnt), C.byref(h)))
        m = cnt.value if cap is None else min(cap, cnt.value)
        st = np.zeros(max(m, 1), dtype=np.int32)
        ix = np.zeros(max(m, 1), dtype=np.int32)
        _check(library().asi_get_flip_log(self.handle, m, _ptr(st), _ptr(ix), C.byref(cnt),
                                          C.byref(h)))
        got = min(m, cnt.value, self.info()["flip_log_capacity"])
        return dict(step=st[:got].copy(), idx=ix[:got].copy(), count=cnt.value, hash=h.value)

    def step_flips(self):
        out = np.zeros(max(self.K, 1), dtype=np.int32)
        _check(library().asi_get_step_flips(self.handle, _ptr(out)))
        return out[:self.K]

    def info(self):
        i = AsiInfo()
        _check(library().asi_get_info(self.handle, C.byref(i)))
        return dict(n=i.n, n_edges=i.n_edges, max_degree=i.max_degree,
                    relax_waves=i.relax_waves, device_bytes=i.device_bytes,
                    field_pass_bytes=i.field_pass_bytes,
                    flip_log_capacity=i.flip_log_capacity)

    def tune(self, sample_steps: int = 20) -> dict:
        """Autotune the relax launch shapes on the next sample_steps steps;
        the state is left exactly as it was."""
        t = AsiTuning()
        _check(library().asi_tune(self.handle, int(sample_steps), C.byref(t)))
        return {name: getattr(t, name) for name, _ in AsiTuning._fields_}

    def tuning(self) -> dict:
        t = AsiTuning()
        _check(library().asi_get_tuning(self.handle, C.byref(t)))
        return {name: getattr(t, name)
                for name in ("relax_waves", "l1_shift", "spec_min", "field_rows")}

    def set_tuning(self, relax_waves: int, l1_shift: int, spec_min: int,
                   field_rows: Optional[int] = None):
        """Set the launch shapes (field_rows None: keep the current one)."""
        if field_rows is None:
            field_rows = self.tuning()["field_rows"]
        t = AsiTuning(relax_waves=int(relax_waves), l1_shift=int(l1_shift), spec_min=int(spec_min),
                      field_rows=int(field_rows))
        _check(library().asi_set_tuning(self.handle, C.byref(t)))

    def set_timing(self, on: bool = True):
        _check(library().asi_set_timing(self.handle, 1 if on else 0))

    def timing(self):
        t = AsiTiming()
        _check(library().asi_get_timing(self.handle, C.byref(t)))
        return dict(field_launches=t.field_launches, field_ms=t.field_ms,
                    relax_launches=t.relax_launches, relax_ms=t.relax_ms)


def switching_rho(a: Sim, b: Sim):
    """Spearman's rho of the switching orders of two instances (Sec. IV.D),
    computed on the device: (rho, (Sab, Saa, Sbb)) with the exact integer
    sums of the rank products."""
    rho = C.c_double(0.0)
    sums = np.zeros(6, dtype=np.int64)
    _check(library().asi_switching_rho(a.handle, b.handle, C.byref(rho), _ptr(sums)))
    tot = tuple(int(np.uint64(sums[2 * c])) + (int(sums[2 * c + 1]) << 64) for c in range(3))
    return rho.value, tot


def switching_rho_noalloc(a: Sim, b: Sim):
    """switching_rho through the allocation-free entry point (static device
    scratch; n <= 2^20, logs <= 2^24 flips)."""
    rho = C.c_double(0.0)
    sums = np.zeros(6, dtype=np.int64)
    _check(library().asi_switching_rho_noalloc(a.handle, b.handle, C.byref(rho), _ptr(sums)))
    tot = tuple(int(np.uint64(sums[2 * c])) + (int(sums[2 * c + 1]) << 64) for c in range(3))
    return rho.value, tot


def batch_run(sims: Sequence[Sim], mode: str = "fused"):
    """Run every instance to the end of its own protocol in batched launches
    (mode: 'lockstep', 'graph' or 'fused', see asi_batch_run)."""
    arr = (C.c_void_p * len(sims))(*[s.handle.value for s in sims])
    flips = np.zeros(len(sims), dtype=np.int64)
    _check(library().asi_batch_run(arr, len(sims), BATCH_MODES[mode], _ptr(flips)))
    return flips


class Server:
    """Continuous-batching server of simulation jobs (device-resident)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, device="hip"):
        self._dev = device if not isinstance(device, str) else make_device(device)
        h = C.c_void_p()
        _check(library().asi_server_create(C.byref(self._dev.struct), int(hbm_budget_bytes),
                                           int(max_slots), C.byref(h)))
        self._h = h
        self._n = {}

    def close(self):
        if getattr(self, "_h", None):
            library().asi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, w, **kw) -> int:
        p, keep = _params(w.xy, w.theta, w.hk, w.spin0, **w.params(), **kw)
        H = np.ascontiguousarray(w.H, dtype=np.float64).reshape(-1, 2)
        jid = C.c_int64(0)
        loc = getattr(w, "h_loc", None)
        sig = getattr(w, "sigma_t", None)
        if loc is None and sig is None:
            _check(library().asi_server_submit(self._h, C.byref(p), len(H), _ptr(H),
                                               C.byref(jid)))
        else:
            if loc is not None:
                loc = np.ascontiguousarray(loc, dtype=np.float64)
                loc = loc[None] if loc.ndim == 2 else loc
                if loc.ndim != 3 or loc.shape[1:] != (len(keep[1]), 2):
                    raise ValueError("h_loc must be (n, 2) or (K, n, 2)")
            if sig is not None:
                sig = np.ascontiguousarray(sig, dtype=np.float64).reshape(-1)
                if len(sig) != len(H):
                    raise ValueError("sigma_t needs one value per protocol step")
            _check(library().asi_server_submit_fields(
                self._h, C.byref(p), len(H), _ptr(H), 0 if loc is None else loc.shape[0],
                _ptr(loc), _ptr(sig), C.byref(jid)))
        self._n[jid.value] = len(keep[1])
        return jid.value

    def step(self, budget_ms: float = 20.0) -> int:
        a = C.c_int32(0)
        _check(library().asi_server_step(self._h, float(budget_ms), C.byref(a)))
        return a.value

    def poll(self, jid: int) -> bool:
        d = C.c_int32(0)
        _check(library().asi_server_poll(self._h, int(jid), C.byref(d)))
        return bool(d.value)

    def take(self, jid: int):
        n = self._n.pop(jid)
        s = np.zeros(n, dtype=np.int8)
        f = C.c_int64(0)
        h = C.c_uint64(0)
        ta = C.c_double(0)
        td = C.c_double(0)
        _check(library().asi_server_take(self._h, int(jid), _ptr(s), C.byref(f), C.byref(h),
                                         C.byref(ta), C.byref(td)))
        return dict(spins=s, flips=f.value, hash=h.value, t_admit=ta.value, t_done=td.value)

    def stats(self) -> dict:
        st = AsiServerStats()
        _check(library().asi_server_get_stats(self._h, C.byref(st)))
        return {name: getattr(st, name) for name, _ in AsiServerStats._fields_}


def load_latency_ns(nbytes: int, hops: int = 100000, lanes: int = 1, seed: int = 1) -> float:
    """Nanoseconds per dependent load (lanes = 1) or per dependent 64-lane
    gather (lanes = 64) over a buffer of nbytes (asi_measure_load_latency)."""
    dev = make_device("hip")
    ns = C.c_double(0.0)
    _check(library().asi_measure_load_latency(C.byref(dev.struct), int(nbytes), int(hops),
                                              int(lanes), int(seed), C.byref(ns)))
    return ns.value
