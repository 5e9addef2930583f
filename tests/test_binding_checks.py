"""The Python binding rejects operands that the kernels would read or write
past their end, before any library call (runs without a GPU: the checks look
only at shapes, strides and dtypes, and the GPU check comes last)."""
import numpy as np
import pytest
import torch

from paper_2303_16999_amd import spmm


def _fake_plan(m=64, k=48, b=16, w="f16", x="f16", y="f16"):
    p = spmm.StaticPlan.__new__(spmm.StaticPlan)
    p.m, p.k, p.b = m, k, b
    p.w, p.x, p.y = spmm.DTYPE_CODES[w], spmm.DTYPE_CODES[x], spmm.DTYPE_CODES[y]
    p.mb, p.kb = -(-m // b), -(-k // b)
    p._h = None
    p._nnzb_cache = 3
    return p


def _raises(fn, text):
    with pytest.raises((ValueError, TypeError)) as ei:
        fn()
    assert text in str(ei.value), str(ei.value)


def test_static_run_rejects_short_or_mistyped_operands():
    p = _fake_plan()
    X = torch.zeros((48, 40), dtype=torch.float16)
    Y = torch.zeros((64, 40), dtype=torch.float16)
    _raises(lambda: p.run(X[:47], Y), "X has 47 rows")
    _raises(lambda: p.run(X, Y[:63]), "Y has 63 rows")
    _raises(lambda: p.run(X, Y.float()), "Y has dtype")
    _raises(lambda: p.run(X.to(torch.bfloat16), Y), "X has dtype")
    _raises(lambda: p.run(X, Y, n=41), "does not fit the 40 columns of X")
    _raises(lambda: p.run(X, Y[:, :16], n=24), "does not fit the 16 columns of Y")
    _raises(lambda: p.run(X.t().contiguous().t(), Y), "unit column stride")
    _raises(lambda: p.run(X[0], Y), "2-D")
    _raises(lambda: p.run(X.numpy(), Y), "torch tensor")
    _raises(lambda: p.run(X, Y, ldx=32), "leading dimension of X")
    # well-formed host tensors pass every check but the last
    _raises(lambda: p.run(X, Y), "X must be a GPU tensor")


def test_fp32_output_plan_needs_fp32_y():
    p = _fake_plan(y="f32")
    X = torch.zeros((48, 8), dtype=torch.float16)
    _raises(lambda: p.run(X, torch.zeros((64, 8), dtype=torch.float16)), "Y has dtype")


def test_set_values_checks_count_and_element_size():
    p = _fake_plan()  # 3 blocks of 16 x 16
    _raises(lambda: p.set_values(torch.zeros(3 * 256 - 1, dtype=torch.float16)), "holds 767 elements")
    _raises(lambda: p.set_values(torch.zeros(3 * 256, dtype=torch.float32)), "4-byte elements")
    _raises(lambda: p.set_values(torch.zeros((3, 16, 32), dtype=torch.float16)[:, :, :16]), "contiguous")
    q = _fake_plan(w="fp8")
    _raises(lambda: q.set_values(torch.zeros(3 * 256, dtype=torch.uint8), torch.zeros(2)), "holds 2 elements")
    _raises(lambda: q.set_values(torch.zeros(3 * 256, dtype=torch.uint8), torch.zeros(3, dtype=torch.float64)),
            "dtype")


def test_dynamic_run_checks_operands():
    h = spmm.DynamicHandle.__new__(spmm.DynamicHandle)
    h.m, h.k, h.b, h.max_nnzb = 64, 64, 16, 8
    h.w = h.x = h.y = spmm.F16
    h._h = None
    i32 = lambda n: torch.zeros(n, dtype=torch.int32)
    X = torch.zeros((64, 8), dtype=torch.float16)
    Y = torch.zeros((64, 8), dtype=torch.float16)
    v = torch.zeros(8 * 256, dtype=torch.float16)
    _raises(lambda: h.run(i32(1), i32(8), i32(8), v, X[:60], Y, i32(1)), "X has 60 rows")
    _raises(lambda: h.run(i32(1), i32(8).long(), i32(8), v, X, Y, i32(1)), "rows has dtype")
    _raises(lambda: h.run(i32(0), i32(8), i32(8), v, X, Y, i32(1)), "nnz_dev holds 0 elements")
    _raises(lambda: h.run(i32(1), i32(8), i32(8), v.float(), X, Y, i32(1)), "values has 4-byte elements")


def test_group_run_checks_every_problem():
    g = spmm.Group.__new__(spmm.Group)
    g._h, g.max_problems = None, 4
    p = _fake_plan()
    X = torch.zeros((48, 8), dtype=torch.float16)
    Y = torch.zeros((64, 8), dtype=torch.float16)
    _raises(lambda: g.run([p, p], [X, X], [Y]), "one entry per problem")
    _raises(lambda: g.run([p, p], [X, X[:10]], [Y, Y]), "X[1] has 10 rows")


def test_serve_submit_checks_host_buffers():
    s = spmm.Server.__new__(spmm.Server)
    s._h, s._keep, s.dims, s._x_bytes, s._y_bytes = None, {}, [64, 128, 64], 2, 2
    x = np.zeros((64, 16), np.float16)
    y = np.zeros((64, 16), np.float16)
    _raises(lambda: s.submit(0, 8, x[:63], y), "x_host has 63 rows")
    _raises(lambda: s.submit(0, 17, x, y), "does not fit the 16 columns of x_host")
    _raises(lambda: s.submit(0, 8, x, y.astype(np.float32)), "y_host has 4-byte elements")
    _raises(lambda: s.submit(0, 8, x[:, ::2], y), "contiguous rows")
