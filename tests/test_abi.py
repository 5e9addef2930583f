"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before touching a GPU (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2303_16999_amd import spmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^(?:spmm_status_t|const char\*)\s+(spmm_\w+)\s*\(", text, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    L = spmm.lib()
    names = _declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
        assert name in spmm.SIGNATURES, name


def _plan(m=64, k=64, b=16, w=spmm.F16, x=spmm.F16, y=spmm.F16, mask=None, opts=None):
    L = spmm.lib()
    if mask is None:
        mask = np.ones((max(1, -(-m // b)) if b > 0 else 1, max(1, -(-k // b)) if b > 0 else 1), np.uint8)
    h = ctypes.c_void_p()
    st = L.spmm_plan_static(m, k, b, mask.ctypes.data_as(ctypes.c_void_p), w, x, y, opts, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("b", [0, 2, 3, 48, 128, -16])
def test_bad_block_size_is_invalid_arg(b):
    st, h = _plan(b=b, mask=np.ones((4, 4), np.uint8))
    assert st == spmm.ERR_INVALID_ARG and not h.value
    assert b"block size" in spmm.lib().spmm_last_error()


@pytest.mark.parametrize("w,x,y", [(spmm.F16, spmm.BF16, spmm.F16), (spmm.F32, spmm.F16, spmm.F32),
                                   (spmm.BF16, spmm.BF16, spmm.F16), (spmm.FP8_E4M3, spmm.F32, spmm.F32),
                                   (7, spmm.F16, spmm.F16)])
def test_unsupported_dtype_triples(w, x, y):
    st, h = _plan(w=w, x=x, y=y)
    assert st == spmm.ERR_UNSUPPORTED and not h.value


def test_bad_sizes_and_null_pointers():
    L = spmm.lib()
    h = ctypes.c_void_p()
    assert L.spmm_plan_static(0, 16, 16, None, 1, 1, 1, None, ctypes.byref(h)) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_static(16, 16, 16, None, 1, 1, 1, None, ctypes.byref(h)) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_static(16, 16, 16, None, 1, 1, 1, None, None) == spmm.ERR_INVALID_ARG
    assert L.spmm_run_static(None, 4, None, 4, None, 4, None) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_set_values(None, None, None, None) == spmm.ERR_INVALID_ARG
    assert L.spmm_dynamic_create(16, 16, 16, -1, 1, 1, 1, None, ctypes.byref(h)) == spmm.ERR_INVALID_ARG
    assert L.spmm_dynamic_create(16, 16, 5, 4, 1, 1, 1, None, ctypes.byref(h)) == spmm.ERR_INVALID_ARG
    assert L.spmm_run_dynamic(None, None, None, None, None, None, 4, None, 4, None, 4, None, None) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_destroy(None) == spmm.OK and L.spmm_dynamic_destroy(None) == spmm.OK
    opts = spmm.PlanOpts(-1, 0, 0, 0)
    mask = np.ones((1, 1), np.uint8)
    assert L.spmm_plan_static(16, 16, 16, mask.ctypes.data_as(ctypes.c_void_p), 1, 1, 1, ctypes.byref(opts),
                              ctypes.byref(h)) == spmm.ERR_INVALID_ARG


def test_binding_raises_with_message():
    with pytest.raises(spmm.SpmmError) as ei:
        spmm.StaticPlan(64, 64, 3, np.ones((22, 22), np.uint8))
    assert ei.value.status == spmm.ERR_INVALID_ARG


def test_plan_variant_option_checked_on_host():
    for variant, b in [(3, 16), (16, 16), (-2, 16), (2, 8), (3 * 256 + 8, 16), (2 + 256, 4)]:
        opts = spmm.PlanOpts(0, 0, 0, variant)
        st, h = _plan(b=b, opts=ctypes.byref(opts))
        assert st == spmm.ERR_INVALID_ARG and not h.value, (variant, b)
        assert b"variant" in spmm.lib().spmm_last_error()


def test_dense_dispatch_option_checked_on_host():
    mask = np.ones((4, 4), np.uint8)
    cases = [((0, 0, 0, 0, 3), spmm.DTYPE_CODES["f16"], spmm.ERR_INVALID_ARG, b"dense_dispatch"),
             ((0, 0, 0, 3 * 256, 0), spmm.DTYPE_CODES["f16"], spmm.ERR_INVALID_ARG, b"dense copy"),
             ((0, 0, 0, 0, 1), spmm.DTYPE_CODES["f32"], spmm.ERR_UNSUPPORTED, b"dense dispatch")]
    for fields, dt, want, msg in cases:
        opts = spmm.PlanOpts(*fields)
        h = ctypes.c_void_p()
        st = spmm.lib().spmm_plan_static(64, 64, 16, mask.ctypes.data_as(ctypes.c_void_p), dt, dt, dt,
                                         ctypes.byref(opts), ctypes.byref(h))
        assert st == want and not h.value, fields
        assert msg in spmm.lib().spmm_last_error(), fields
    assert spmm.lib().spmm_plan_dispatch(None, None, None) == spmm.ERR_INVALID_ARG


def test_autotune_and_group_reject_bad_arguments():
    L = spmm.lib()
    v = ctypes.c_int32()
    assert L.spmm_autotune_static(None, 64, None, 64, None, 64, None, ctypes.byref(v), None) == spmm.ERR_INVALID_ARG
    vs, ts = (ctypes.c_int32 * 8)(), (ctypes.c_float * 8)()
    cnt = ctypes.c_int32()
    assert L.spmm_autotune_static_all(None, 64, None, 64, None, 64, None, 8, vs, ts, ctypes.byref(cnt),
                                      None) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_variant(None, 64, ctypes.byref(v)) == spmm.ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert L.spmm_group_create(0, ctypes.byref(h)) == spmm.ERR_INVALID_ARG and not h.value
    assert L.spmm_group_create(4, None) == spmm.ERR_INVALID_ARG
    assert L.spmm_group_run(None, 1, None, None, None, None, None, None, None, None) == spmm.ERR_INVALID_ARG
    assert L.spmm_group_destroy(None) == spmm.OK


def test_b64_needs_16bit_x():
    st, h = _plan(m=128, k=128, b=64, w=spmm.F32, x=spmm.F32, y=spmm.F32, mask=np.ones((2, 2), np.uint8))
    assert st == spmm.ERR_UNSUPPORTED and not h.value
    assert b"b = 64" in spmm.lib().spmm_last_error()


def _ell(cols, m=64, k=64, b=16):
    cols = np.ascontiguousarray(np.asarray(cols, np.int32))
    h = ctypes.c_void_p()
    st = spmm.lib().spmm_plan_ell(m, k, b, cols.shape[1], cols.ctypes.data_as(ctypes.c_void_p), spmm.F16, spmm.F16,
                                  spmm.F16, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("cols", [[[0, 4], [1, -1], [2, 3], [0, 1]],      # column 4 is outside kb = 4
                                  [[0, -2], [1, -1], [2, 3], [0, 1]],     # -2 is not the empty marker
                                  [[1, 1], [1, -1], [2, 3], [0, 1]]])     # column twice in a row
def test_ell_rejects_bad_patterns_before_touching_the_device(cols):
    st, h = _ell(cols)
    assert st == spmm.ERR_INVALID_ARG and not h.value


def test_ell_rejects_null_and_negative_width():
    h = ctypes.c_void_p()
    L = spmm.lib()
    assert L.spmm_plan_ell(64, 64, 16, 2, None, spmm.F16, spmm.F16, spmm.F16, None, ctypes.byref(h)) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_ell(64, 64, 16, -1, None, spmm.F16, spmm.F16, spmm.F16, None, ctypes.byref(h)) == spmm.ERR_INVALID_ARG
    assert L.spmm_plan_set_values_ell(None, None, None, None) == spmm.ERR_INVALID_ARG
