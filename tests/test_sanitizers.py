"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

1. The tier-1 oracle (oracle/relax.cpp) built with g++ -fsanitize=address,
   undefined runs small whole protocols (square 10 x 10, a random cloud
   with thermal noise and a local field, an annealing schedule) in a child
   process and must reproduce the plain build's flip counts and checksums
   with no sanitizer report.
2. The library's host code (asi_runtime.hip) built with the sanitizers on
   the host side only runs its argument validation -- every rejected
   asi_create, the limits of asi_measure_load_latency and the NULL-handle
   paths -- in a child process: each call must return its error status,
   before any device call, with no sanitizer report.

Device code is built as usual (sanitizers are host-only here).
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _run_child(code, preload, extra_env=None, timeout=600):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=87"
    env["PYTHONPATH"] = ROOT
    env.update(extra_env or {})
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=timeout)
    report = r.stderr + r.stdout
    assert "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert "runtime error:" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liborc_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-std=c++17", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "relax.cpp"),
                           "-o", lib])
    asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    code = f"""
        import json
        import numpy as np
        from oracle import native as N
        from paper_2002_11401_amd import workloads as W

        def cases():
            yield W.square_10x10_triangle()
            xy, th = W.random_cloud(300, 5)
            n = len(th)
            H = W.rotating(60, 0.3, 40)
            w = W.Workload("cloud300", xy, th, W.polarised_spins(th, H[0]),
                           W.disorder_hk(n, 0.2, 0.05, 3), H, alpha=0.01,
                           neighbor_distance=3.0, b=0.38, c=1.0, beta=1.5, gamma=3.9,
                           thermal_std=0.01, thermal_seed=4)
            w.h_loc = W.random_local(n, 1, 0.02, 8)
            yield w
            yield W.square_anneal(side=8, n_steps=40)

        def run_all():
            out = []
            for w in cases():
                o = N.Oracle.from_workload(w)
                o.set_spins(w.spin0)
                r = o.run(w.H)
                out.append((w.name, int(r["n_flips"]), str(r["hash"])))
                o.close()
            return out

        plain = run_all()
        N.LIB = {lib!r}
        N._lib = None
        san = run_all()
        print(json.dumps(dict(plain=plain, san=san)))
        assert plain == san, (plain, san)
        assert all(f > 0 for _, f, _ in san)
    """
    out = _run_child(code, asan)
    assert '"san"' in out


def test_library_validation_under_asan_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    lib = str(tmp_path / "libasi_san.so")
    csrc = os.path.join(ROOT, "paper_2002_11401_amd", "csrc")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                           "-shared", "-ffp-contract=off", "-Xclang", "-target-feature",
                           "-Xclang", "-packed-fp32-ops", "-fno-omit-frame-pointer",
                           "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(csrc, "asi_kernels.hip"),
                           os.path.join(csrc, "asi_runtime.hip"),
                           "-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx",
                           "-o", lib], stderr=subprocess.DEVNULL)
    asan = subprocess.check_output([os.path.join(ROCM, "llvm", "bin", "clang++"),
                                    "-print-file-name=libclang_rt.asan-x86_64.so"],
                                   text=True).strip()
    code = """
        import ctypes as C
        import math
        import numpy as np
        from paper_2002_11401_amd import asi

        L = asi.library()
        assert asi.LIB_PATH.endswith("libasi_san.so"), asi.LIB_PATH
        n = 12
        xy = np.random.default_rng(1).uniform(0, 10, (n, 2))
        th = np.zeros(n)
        good = dict(xy=xy, theta=th, alpha=0.001, neighbor_distance=2.0, b=1.0, c=1.0,
                    beta=3.0, gamma=3.0, hk_mean=0.2)

        def params(**kw):
            a = dict(good)
            a.update(kw)
            keep = []
            p = asi.AsiParams()
            p.struct_size = C.sizeof(asi.AsiParams)
            p.n = a.pop("n", n)
            for name in ("xy", "theta", "hk", "spin0"):
                v = a.pop(name, None)
                if v is None:
                    setattr(p, name, None)
                else:
                    arr = np.ascontiguousarray(v, dtype=np.int8 if name == "spin0" else np.float64)
                    keep.append(arr)
                    setattr(p, name, arr.ctypes.data)
            for k, v in a.items():
                setattr(p, k, v)
            return p, keep

        bad = [dict(n=0), dict(xy=None), dict(theta=None), dict(hk_mean=0.0),
               dict(k_disorder=-1.0), dict(alpha=math.inf), dict(neighbor_distance=-1.0),
               dict(b=0.0), dict(c=-1.0), dict(beta=math.nan), dict(gamma=math.inf),
               dict(thermal_std=-0.1), dict(max_flips_per_step=-1),
               dict(flip_log_capacity=-5), dict(field_mode=3),
               dict(xy=np.full((n, 2), math.nan)), dict(theta=np.full(n, math.inf)),
               dict(hk=np.full(n, -0.2)), dict(spin0=np.full(n, 2))]
        for kw in bad:
            p, keep = params(**kw)
            h = C.c_void_p()
            st = L.asi_create(C.byref(p), None, C.byref(h))
            assert st == asi.ASI_EINVAL, (kw, st)
            assert h.value is None
            msg = L.asi_last_error().decode()
            assert msg, kw
        p, keep = params()
        p.struct_size = 8
        h = C.c_void_p()
        assert L.asi_create(C.byref(p), None, C.byref(h)) == asi.ASI_EINVAL
        assert L.asi_create(None, None, C.byref(h)) == asi.ASI_EINVAL
        assert L.asi_create(C.byref(p), None, None) == asi.ASI_EINVAL
        # calls on a NULL handle fail cleanly
        f = C.c_int64()
        assert L.asi_run(None, 0, 1, C.byref(f)) == asi.ASI_EINVAL
        assert L.asi_relax(None, C.byref(f)) == asi.ASI_EINVAL
        assert L.asi_get_state(None, None, None, None, None) == asi.ASI_EINVAL
        assert L.asi_destroy(None) == asi.ASI_OK
        # latency probe limits are checked before any device call
        ns = C.c_double()
        for args in ((1 << 20, 0, 1), (1 << 20, 10, 0), (1 << 20, 10, 65), (1024, 10, 1)):
            assert L.asi_measure_load_latency(None, *args, 7, C.byref(ns)) == asi.ASI_EINVAL
        print("validation ok", len(bad))
    """
    out = _run_child(code, asan, {"ASI_LIBRARY": lib})
    assert "validation ok" in out
