"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2002_11401_amd import asi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "asi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(asi_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = asi.library()
    names = _declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(asi.SIGNATURES), set(names) ^ set(asi.SIGNATURES)


def test_struct_layouts_match_header():
    # asi_params: u32 + pad, i64, 4 pointers, 8 doubles, u64, 2 x i64
    assert C.sizeof(asi.AsiParams) == 8 + 8 + 4 * 8 + 7 * 8 + 8 + 8 + 8 + 8 + 3 * 8
    assert C.sizeof(asi.AsiDevice) == 4 * 8
    assert C.sizeof(asi.AsiInfo) == 8 + 8 + 4 + 4 + 8 + 8 + 8
    assert C.sizeof(asi.AsiServerStats) == 4 * 8 + 4 * 8
    assert C.sizeof(asi.AsiTuning) == 4 + 4 + 8 + 8 + 8 + 4 + 4


def test_invalid_arguments_fail_before_touching_the_device():
    lib = asi.library()
    h = C.c_void_p()
    assert lib.asi_create(None, None, C.byref(h)) == asi.ASI_EINVAL
    assert b"NULL" in lib.asi_last_error()
    p, keep = asi._params([[0.0, 0.0]], [0.0], [-0.2], None, 0.001, 1.0, 1, 1, 3, 3)
    assert lib.asi_create(C.byref(p), None, C.byref(h)) == asi.ASI_EINVAL
    assert b"hk" in lib.asi_last_error()
    p, keep = asi._params([[0.0, 0.0]], [0.0], [0.2], None, 0.001, 1.0, 0.0, 1, 3, 3)
    assert lib.asi_create(C.byref(p), None, C.byref(h)) == asi.ASI_EINVAL
    p, keep = asi._params([[0.0, 0.0]], [0.0], [0.2], [3], 0.001, 1.0, 1, 1, 3, 3)
    assert lib.asi_create(C.byref(p), None, C.byref(h)) == asi.ASI_EINVAL
    p.struct_size = 8
    assert lib.asi_create(C.byref(p), None, C.byref(h)) == asi.ASI_EINVAL
    assert lib.asi_run(None, 0, 1, None) == asi.ASI_EINVAL
    assert lib.asi_destroy(None) == asi.ASI_OK
    assert lib.asi_batch_run(None, 0, 0, None) == asi.ASI_EINVAL
    assert lib.asi_server_get_stats(None, None) == asi.ASI_EINVAL
    assert lib.asi_tune(None, 10, None) == asi.ASI_EINVAL
    assert lib.asi_get_tuning(None, None) == asi.ASI_EINVAL
    assert lib.asi_set_tuning(None, None) == asi.ASI_EINVAL
    assert lib.asi_set_local_field(None, 1, None) == asi.ASI_EINVAL
    assert lib.asi_set_thermal_schedule(None, 1, None) == asi.ASI_EINVAL
    assert lib.asi_set_local_wave(None, None, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0) == asi.ASI_EINVAL
    assert lib.asi_magnetization(None, None) == asi.ASI_EINVAL
    assert lib.asi_group_magnetization(None, 1, None, None, None) == asi.ASI_EINVAL
    assert lib.asi_spin_correlation(None, None, 1.0, 4, None, None) == asi.ASI_EINVAL
    assert lib.asi_set_magnetization_log(None, 1) == asi.ASI_EINVAL
    assert lib.asi_get_magnetization_log(None, None) == asi.ASI_EINVAL
    assert lib.asi_server_step(None, 1.0, None) == asi.ASI_EINVAL
    assert lib.asi_server_submit_fields(None, None, 1, None, 0, None, None,
                                        None) == asi.ASI_EINVAL
    assert lib.asi_server_destroy(None) == asi.ASI_OK


def test_flip_hash_definition():
    # hash of an empty log is the FNV offset basis; one entry by hand
    assert asi.flip_hash([], []) == 0xcbf29ce484222325
    w = (3 << 32) | 7
    assert asi.flip_hash([3], [7]) == ((0xcbf29ce484222325 ^ w) * 0x100000001b3) % 2 ** 64
