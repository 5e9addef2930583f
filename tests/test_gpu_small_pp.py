"""The software-pipelined MFMA form of the b = 4 / 8 kernel against the plain
one, bit for bit, and the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import TOL, Case, dev, stored_f64, y_f64

pytestmark = pytest.mark.gpu


def _static(c, pp, monkeypatch):
    monkeypatch.setenv("SPMM_SMALL_PP", "1" if pp else "0")
    monkeypatch.setenv("SPMM_SMALL_LDS", "0")  # the kernel without LDS, whose two forms these tests compare
    plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y)
    vals, X, scales = c.device_inputs()
    plan.set_values(vals, scales)
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    return Y


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "f32"), ("bf16", "bf16")])
@pytest.mark.parametrize("b", [4, 8])
def test_small_pp_equals_plain_and_oracle(w, y, b, monkeypatch):
    # ragged m, k and n; d = 0.45 over 180 block columns: rows of about 81 blocks
    # (more than one 64-block chunk, counts not multiples of 32 / b)
    c = Case(b * 37 + b // 2 + 1, b * 180 - 3, 203, b, 0.45, w=w, y=y, seed=70 + b)
    assert c.mask.sum(1).max() > 64
    Yp = _static(c, True, monkeypatch)
    Yr = _static(c, False, monkeypatch)
    assert torch.equal(Yp[:, : c.n], Yr[:, : c.n])
    assert O.rel_fro(y_f64(Yp, c), c.oracle()) <= TOL[y]


@pytest.mark.parametrize("b", [4, 8])
def test_small_pp_short_and_empty_rows(b, monkeypatch):
    bpm = 32 // b
    mb, kb = 3 * bpm + 2, 2 * bpm + 5
    mask = np.zeros((mb, kb), np.uint8)
    for r in range(mb):
        mask[r, : r % (bpm + 3)] = 1  # 0 .. bpm + 2 blocks per row
    c = Case(mb * b, kb * b, 136, b, 0.0, w="f16", seed=5, mask=mask)
    Yp = _static(c, True, monkeypatch)
    Yr = _static(c, False, monkeypatch)
    assert torch.equal(Yp[:, : c.n], Yr[:, : c.n])
    got = y_f64(Yp, c)
    assert not np.isnan(got).any()
    assert O.rel_fro(got, c.oracle()) <= TOL["f16"]


def test_small_pp_integer_data_bit_exact(monkeypatch):
    c = Case(8 * 256, 8 * 256, 256, 8, 1 / 8, w="bf16", seed=9, integer=True)
    ref = c.oracle()
    assert np.abs(ref).max() <= 256
    assert np.array_equal(y_f64(_static(c, True, monkeypatch), c), ref)


@pytest.mark.parametrize("b", [4, 8])
def test_small_pp_dynamic_equals_plain(b, monkeypatch):
    mb, kb, n = 512 // b * 4, 512 // b * 4, 256
    max_nnz = min(8000, mb * kb // 8)
    rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=80 + b, dtype="f16")
    pad = max_nnz - len(rows)
    r = dev(np.concatenate([rows, np.zeros(pad, np.int32)]))
    cc = dev(np.concatenate([cols, np.zeros(pad, np.int32)]))
    v = dev(np.concatenate([vals, np.zeros((pad, b, b), vals.dtype)]))
    nnz = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    Xs = synth.to_storage(synth.normal((kb * b, n), 81), "f16")
    h = spmm.DynamicHandle(mb * b, kb * b, b, max_nnz, "f16")
    outs = []
    monkeypatch.setenv("SPMM_SMALL_LDS", "0")
    for pp in ("1", "0"):
        monkeypatch.setenv("SPMM_SMALL_PP", pp)
        Y = torch.full((mb * b, n), float("nan"), dtype=torch.float16, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, cc, v, dev(Xs), Y, status)
        torch.cuda.synchronize()
        assert status.item() == 0
        outs.append(Y)
    assert torch.equal(outs[0], outs[1])
    ref = O.spmm_blockwise(mb * b, kb * b, b, rows, cols, synth.storage_to_f64(vals, "f16"),
                           synth.storage_to_f64(Xs, "f16"))
    assert O.rel_fro(stored_f64(outs[0], "f16"), ref) <= TOL["f16"]
