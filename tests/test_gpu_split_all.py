"""Every block row split over a workgroup's four waves (b = 16): the form the
rule takes for launches too small to fill the chip with one wave per row, and
autotuner candidate 4 * 256. Against the FP64 oracle within the rounding bound,
deterministic, integer data exact, equal to the grouped launch and to the
dynamic call that take the same form."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import TOL, Case, assert_elementwise, dev, round_like, y_f64

pytestmark = pytest.mark.gpu


def _run(c, monkeypatch, split, variant=0):
    monkeypatch.setenv("SPMM_AUTOTUNE", "0")
    if split is None:
        monkeypatch.delenv("SPMM_SPLIT_ALL", raising=False)
    else:
        monkeypatch.setenv("SPMM_SPLIT_ALL", "1" if split else "0")
    plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y, variant=variant)
    vals, X, _ = c.device_inputs()
    plan.set_values(vals)
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    return plan, Y


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "f32"), ("bf16", "bf16")])
@pytest.mark.parametrize("n", [1, 70, 300])
def test_split_all_matches_oracle(w, y, n, monkeypatch):
    # ragged m and k, rows from 0 to ~40 blocks
    c = Case(16 * 37 + 5, 16 * 90 + 7, n, 16, 0.3, w=w, y=y, seed=600 + n)
    _, Y = _run(c, monkeypatch, True)
    got, ref = y_f64(Y, c), c.oracle()
    assert O.rel_fro(got, ref) <= TOL[y]
    assert_elementwise(got, ref, c.abs_oracle(), c.k, y)
    assert torch.isnan(Y[:, c.n:].float()).all().item()
    _, Y2 = _run(c, monkeypatch, True)
    assert torch.equal(Y[:, : c.n], Y2[:, : c.n])  # deterministic
    _, Y3 = _run(c, monkeypatch, None, variant=4 * 256)  # the same form through the variant
    assert torch.equal(Y[:, : c.n], Y3[:, : c.n])


def test_split_all_integer_data_exact_and_empty_rows(monkeypatch):
    mask = synth.block_mask(40, 60, 0.4, 7)
    mask[3:9] = 0
    c = Case(16 * 40, 16 * 60, 96, 16, 0.0, w="bf16", seed=610, integer=True, mask=mask)
    _, Y = _run(c, monkeypatch, True)
    assert np.array_equal(y_f64(Y, c), round_like(c.oracle(), "bf16"))
    assert torch.all(Y[3 * 16: 9 * 16, : c.n] == 0).item()


def test_rule_splits_small_launches_and_group_follows(monkeypatch):
    # m = 1024, n = 64: 16 row quads x 1 tile, rows of ~32 blocks: the rule splits
    c = Case(1024, 2048, 64, 16, 1 / 4, w="f16", seed=620)
    _, Ys = _run(c, monkeypatch, True)
    _, Yr = _run(c, monkeypatch, None)
    assert torch.equal(Ys[:, : c.n], Yr[:, : c.n])
    _, Yu = _run(c, monkeypatch, False)
    assert O.rel_fro(y_f64(Yu, c), y_f64(Ys, c)) <= 1e-3
    # the grouped launch takes the same form for the same problem
    monkeypatch.delenv("SPMM_SPLIT_ALL", raising=False)
    plan, Y1 = _run(c, monkeypatch, None)
    _, X, _ = c.device_inputs()
    Yg = c.new_Y()
    spmm.Group(4).run([plan], [X], [Yg], ns=[c.n])
    torch.cuda.synchronize()
    assert torch.equal(Yg[:, : c.n], Y1[:, : c.n])


def test_dynamic_call_splits_like_static(monkeypatch):
    monkeypatch.setenv("SPMM_AUTOTUNE", "0")
    monkeypatch.delenv("SPMM_SPLIT_ALL", raising=False)
    b, mb, kb, n = 16, 128, 256, 256
    max_nnz = mb * kb // 8
    rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=630, dtype="f16", lo_frac=1.0)
    M = np.zeros((mb, kb), np.uint8)
    M[rows, cols] = 1
    order = np.lexsort((cols, rows))
    plan = spmm.StaticPlan(mb * b, kb * b, b, M, "f16", variant=8)  # width of the dynamic rule, form by rule
    plan.set_values(dev(np.ascontiguousarray(vals[order])))
    X = dev(synth.to_storage(synth.normal((kb * b, n), 631), "f16"))
    Ys = torch.empty((mb * b, n), dtype=torch.float16, device="cuda")
    plan.run(X, Ys)
    h = spmm.DynamicHandle(mb * b, kb * b, b, max_nnz, "f16")
    pad = max_nnz - len(rows)
    r = dev(np.concatenate([rows, np.zeros(pad, np.int32)]))
    cc = dev(np.concatenate([cols, np.zeros(pad, np.int32)]))
    v = dev(np.concatenate([vals, np.zeros((pad, b, b), vals.dtype)]))
    nnz = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    Yd = torch.empty_like(Ys)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, cc, v, X, Yd, st)
    torch.cuda.synchronize()
    assert st.item() == 0
    assert torch.equal(Ys, Yd)
    ref = O.spmm_blockwise(mb * b, kb * b, b, rows, cols, synth.storage_to_f64(vals, "f16"),
                           synth.storage_to_f64(synth.to_storage(synth.normal((kb * b, n), 631), "f16"), "f16"))
    assert O.rel_fro(Yd.cpu().numpy().astype(np.float64), ref) <= TOL["f16"]
