"""The software-pipelined row-wise kernel (launches of at most two workgroups
per CU) against the plain row-wise kernel, bit for bit, and the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import TOL, Case, dev, stored_f64, y_f64

pytestmark = pytest.mark.gpu


def _static(c, variant, pp, monkeypatch):
    monkeypatch.setenv("SPMM_ROW_PP", "1" if pp else "0")
    plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y, variant=variant)
    vals, X, scales = c.device_inputs()
    plan.set_values(vals, scales)
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    return Y


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "f32"), ("bf16", "bf16"), ("f16", "f32")])
@pytest.mark.parametrize("variant", [2, 4, 8])
@pytest.mark.parametrize("b", [16, 32])
def test_pp_equals_row_kernel_and_oracle(w, y, variant, b, monkeypatch):
    # ragged m, k and n; d = 0.45 over 150 block columns gives rows of about 67
    # blocks (more than one 64-block chunk, odd and even counts)
    c = Case(b * 37 + 5, b * 150 - 3, 203, b, 0.45, w=w, y=y, seed=61 + variant)
    assert c.mask.sum(1).max() > 64
    Yp = _static(c, variant, True, monkeypatch)
    Yr = _static(c, variant, False, monkeypatch)
    assert torch.equal(Yp[:, : c.n], Yr[:, : c.n])
    assert O.rel_fro(y_f64(Yp, c), c.oracle()) <= TOL[y]


def test_pp_empty_rows_and_single_blocks(monkeypatch):
    # rows with 0, 1, 2 and 3 blocks; NaN-prefilled Y must be fully overwritten
    mb, kb = 12, 9
    mask = np.zeros((mb, kb), np.uint8)
    for r in range(mb):
        mask[r, : r % 4] = 1
    c = Case(mb * 16, kb * 16, 40, 16, 0.0, w="f16", seed=3, mask=mask)
    Yp = _static(c, 8, True, monkeypatch)
    Yr = _static(c, 8, False, monkeypatch)
    assert torch.equal(Yp[:, : c.n], Yr[:, : c.n])
    got = y_f64(Yp, c)
    assert not np.isnan(got).any()
    assert O.rel_fro(got, c.oracle()) <= TOL["f16"]
    assert not got[0:16].any() and not got[64:80].any()  # rows without blocks are +0


def test_pp_integer_data_bit_exact(monkeypatch):
    c = Case(16 * 64, 16 * 64, 256, 16, 1 / 8, w="f16", seed=7, integer=True)
    ref = c.oracle()
    assert np.abs(ref).max() <= 2048
    Yp = _static(c, 8, True, monkeypatch)
    assert np.array_equal(y_f64(Yp, c), ref)


@pytest.mark.parametrize("w,b", [("f16", 16), ("bf16", 16), ("bf16", 32)])
def test_pp_dynamic_equals_row_kernel(w, b, monkeypatch):
    # b = 16: the dynamic benchmark's shape, 256 x 256 blocks, n = 512, up to
    # 8192 blocks; b = 32: 96 x 80 blocks, up to 1920
    mb, kb, n = (256, 256, 512) if b == 16 else (96, 80, 512)
    max_nnz = mb * kb // 8 if b == 16 else mb * kb // 4
    rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=44, dtype="f16")
    vals = synth.to_storage(synth.storage_to_f64(vals, "f16"), w)
    pad = max_nnz - len(rows)
    r = dev(np.concatenate([rows, np.zeros(pad, np.int32)]))
    c = dev(np.concatenate([cols, np.zeros(pad, np.int32)]))
    v = dev(np.concatenate([vals, np.zeros((pad, b, b), vals.dtype)]))
    nnz = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    Xs = synth.to_storage(synth.normal((kb * b, n), 45), w)
    X = dev(Xs)
    h = spmm.DynamicHandle(mb * b, kb * b, b, max_nnz, w)
    outs = []
    for pp in ("1", "0"):
        monkeypatch.setenv("SPMM_ROW_PP", pp)
        Y = torch.full((mb * b, n), float("nan"), dtype=X.dtype, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == 0
        outs.append(Y)
    assert torch.equal(outs[0], outs[1])
    cs = np.random.default_rng(46).choice(n, 64, replace=False)
    ref = O.spmm_blockwise_columns(mb * b, kb * b, b, rows, cols, synth.storage_to_f64(vals, w),
                                   synth.storage_to_f64(Xs, w), cs)
    assert O.rel_fro(stored_f64(outs[0][:, torch.from_numpy(cs).cuda()], w), ref) <= TOL[w]


def test_pp_default_choice_follows_the_grid(monkeypatch):
    """Without the override both launch shapes give the plain kernel's result."""
    monkeypatch.delenv("SPMM_ROW_PP", raising=False)
    # the pipelined kernel: 16 workgroups with rows of 16 blocks (m = 1024, n = 64,
    # d = 1/4); the plain one: rows of 4 blocks (d = 1/16), and 1024 workgroups
    # (m = 4096, n = 2048)
    for m, n, d in ((1024, 64, 1 / 4), (1024, 64, 1 / 16), (4096, 2048, 1 / 16)):
        c = Case(m, m, n, 16, d, w="f16", seed=n)
        plan = spmm.StaticPlan(c.m, c.k, 16, c.mask, "f16")
        vals, X, _ = c.device_inputs()
        plan.set_values(vals)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        Yr = _static(c, 0, False, monkeypatch)
        monkeypatch.delenv("SPMM_ROW_PP", raising=False)
        assert torch.equal(Y[:, : c.n], Yr[:, : c.n])
