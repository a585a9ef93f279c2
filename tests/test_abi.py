"""The C-ABI library loads, exports every symbol include/lbp.h declares, and
rejects malformed input before touching the device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbp_[a-z_0-9]+)\s*\(", text)))


def _lib():
    from paper_2605_00038_amd import _lib as L
    return L, L.load()


def test_header_symbols_exported():
    L, lib = _lib()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.SIGNATURES)


def test_params_struct_layout_and_defaults():
    L, lib = _lib()
    assert ctypes.sizeof(L.Params) == 48
    p = L.Params()
    lib.lbp_params_default(ctypes.byref(p))
    assert (p.max_iter, p.msg, p.lottery, p.lottery_skip, p.osd, p.osd_order) == (100, L.MSG_INT8, 1, 6, L.OSD_0, 10)
    assert lib.lbp_version() >= 100


def _create(m, n, rp, ci, p):
    L, lib = _lib()
    h = ctypes.c_void_p()
    rp = np.asarray(rp, np.int32)
    ci = np.asarray(ci, np.int32)
    p = np.asarray(p, np.float64)
    st = lib.lbp_code_create(m, n, rp.ctypes.data, ci.ctypes.data, p.ctypes.data, ctypes.byref(h))
    return st, lib.lbp_last_error().decode()


@pytest.mark.parametrize("case,expect", [
    (dict(m=2, n=3, rp=[0, 2, 2], ci=[0, 1], p=[0.1] * 3), -1),           # empty row
    (dict(m=1, n=3, rp=[0, 2], ci=[1, 1], p=[0.1] * 3), -1),              # duplicate column
    (dict(m=1, n=3, rp=[0, 2], ci=[2, 1], p=[0.1] * 3), -1),              # unsorted
    (dict(m=1, n=3, rp=[0, 2], ci=[0, 3], p=[0.1] * 3), -1),              # out of range
    (dict(m=1, n=3, rp=[0, 2], ci=[0, 1], p=[0.1, 0.0, 0.1]), -1),        # prior 0
    (dict(m=1, n=3, rp=[0, 2], ci=[0, 1], p=[0.1, 1.0, 0.1]), -1),        # prior 1
    (dict(m=1, n=3, rp=[0, 2], ci=[0, 1], p=[0.1, float("nan"), 0.1]), -1),
    (dict(m=1, n=10, rp=[0, 9], ci=list(range(9)), p=[0.1] * 10), -6),    # row weight 9
    (dict(m=0, n=3, rp=[0], ci=[], p=[0.1] * 3), -1),
])
def test_code_create_rejects(case, expect):
    st, msg = _create(case["m"], case["n"], case["rp"], case["ci"], case["p"])
    assert st == expect
    assert msg


def test_null_handles_are_rejected():
    L, lib = _lib()
    p = L.Params()
    lib.lbp_params_default(ctypes.byref(p))
    h = ctypes.c_void_p()
    assert lib.lbp_decoder_create(None, ctypes.byref(p), 10, ctypes.byref(h)) == L.LBP_EINVAL
    assert lib.lbp_decode(None, 1, 0, None, None, None, None, None, None) == L.LBP_EINVAL
    assert lib.lbp_decode_host(None, 1, 0, None, None, None, None, None) == L.LBP_EINVAL
    assert lib.lbp_decoder_set_osd_capacity(None, 5) == L.LBP_EINVAL
    assert lib.lbp_decoder_osd_capacity(None) == 0
    assert "NULL" in lib.lbp_last_error().decode()


def test_server_and_keyed_calls_reject_bad_arguments_before_device_use():
    L, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.lbp_server_create(0, 0, ctypes.byref(h)) == L.LBP_EINVAL      # max_slots < 1
    assert lib.lbp_server_create(0, 65, ctypes.byref(h)) == L.LBP_EINVAL     # max_slots > 64
    assert lib.lbp_server_create(-1, 4, ctypes.byref(h)) == L.LBP_EINVAL     # negative budget
    assert lib.lbp_server_create(0, 4, None) == L.LBP_EINVAL
    slot = ctypes.c_int32()
    t = ctypes.c_uint64()
    p = L.Params()
    lib.lbp_params_default(ctypes.byref(p))
    assert lib.lbp_server_add_code(None, None, ctypes.byref(p), ctypes.byref(slot)) == L.LBP_EINVAL
    assert lib.lbp_server_submit(None, 0, 1, 0, 0, None, ctypes.byref(t)) == L.LBP_EINVAL
    assert lib.lbp_server_poll(None, 1, None, None, None) == L.LBP_EINVAL
    assert lib.lbp_server_wait(None, 1, 0, None, None, None) == L.LBP_EINVAL
    assert lib.lbp_server_cancel(None, 1) == L.LBP_EINVAL
    assert lib.lbp_server_slot_info(None, 0, None, None, None, None, None) == L.LBP_EINVAL
    assert lib.lbp_server_run_load(None, 1, None, None, None, 1, 1, 0.0, 0, None, None, None) == L.LBP_EINVAL
    lib.lbp_server_destroy(None)
    assert lib.lbp_decode_keyed(None, 1, None, None, None, None, None, None, None) == L.LBP_EINVAL
    assert lib.lbp_decoder_device_bytes(None) == 0
    assert lib.lbp_decoder_max_batch(None) == 0
