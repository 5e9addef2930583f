"""GPU parity of the small-block path (b = 1, 4, 8) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import plan_ref
from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import assert_elementwise, TOL, Case, dev, round_like, y_f64

pytestmark = pytest.mark.gpu

SMALL = [1, 4, 8]


def _err(case, Y, cols=None):
    ref = case.oracle(cols)
    got = y_f64(Y, case) if cols is None else y_f64(Y, case)[:, cols]
    assert np.all(np.isfinite(got)), "non-finite output"
    return O.rel_fro(got, ref)


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "bf16"), ("f16", "f32"), ("bf16", "f32"), ("f32", "f32")])
@pytest.mark.parametrize("b", SMALL)
@pytest.mark.parametrize("n", [200, 700])  # 256-column tiles, 512-column tiles with a tail
def test_small_ragged_shapes_all_dtypes(w, y, b, n):
    m, k = 37 * b + (b - 1) // 2 + 1, 29 * b + b // 2
    c = Case(m, k, n, b, 0.3, w=w, y=y, seed=31 + b)
    _, Y = c.run_static()
    tol = 1e-5 if w == "f32" else TOL[y if y != "f32" else w]
    assert _err(c, Y) <= tol


@pytest.mark.parametrize("x,y", [("f16", "f16"), ("bf16", "f32")])
@pytest.mark.parametrize("b", SMALL)
def test_small_fp8_block_scales(x, y, b):
    c = Case(41 * b, 23 * b + (b > 1), 333, b, 0.35, w="fp8", x=x, y=y, seed=5, scaled=True)
    _, Y = c.run_static()
    assert _err(c, Y) <= 5e-3


@pytest.mark.parametrize("w", ["f16", "bf16", "f32", "fp8"])
@pytest.mark.parametrize("b", SMALL)
def test_small_integer_data_bit_exact(w, b):
    c = Case(20 * b + 1, 30 * b, 530, b, 0.25, w=w, seed=7, integer=True)
    _, Y = c.run_static()
    ref = c.oracle()
    assert np.abs(ref).max() <= 256
    assert np.array_equal(y_f64(Y, c), round_like(ref, c.y))


@pytest.mark.parametrize("b", SMALL)
def test_small_identity_permutation_bit_exact(b):
    nb, n = 96 // b + 3, 260
    perm = np.random.default_rng(b).permutation(nb)
    mask = np.zeros((nb, nb), np.uint8)
    mask[np.arange(nb), perm] = 1
    c = Case(nb * b, nb * b, n, b, 0.0, w="f16", seed=2, mask=mask)
    eye = np.stack([np.eye(b, dtype=np.float32)] * nb)
    c.vals_store = synth.to_storage(eye, "f16")
    c.vals64 = synth.storage_to_f64(c.vals_store, "f16")
    _, Y = c.run_static()
    expect = np.concatenate([c.X64[col * b:(col + 1) * b] for col in perm])
    assert np.array_equal(y_f64(Y, c), expect)


@pytest.mark.parametrize("b", SMALL)
def test_small_long_rows_and_empty_rows(b):
    # rows longer than one 64-entry chunk (b = 1), empty rows, dense rows
    mb, kb = 12, 300 // b
    mask = synth.block_mask(mb, kb, 0.4, seed=3)
    mask[2] = 0
    mask[5] = 1
    c = Case(mb * b, kb * b, 96, b, 0.0, w="bf16", seed=3, mask=mask)
    _, Y = c.run_static()
    assert _err(c, Y) <= 5e-3
    assert torch.all(Y[2 * b:3 * b, :96] == 0).item()


@pytest.mark.parametrize("b", SMALL)
def test_small_plan_bit_exact_vs_oracle(b):
    mb, kb = 8192 // b // 8, 8192 // b // 8
    mask = synth.block_mask(mb, kb, 1 / 16, seed=b)
    plan = spmm.StaticPlan(mb * b, kb * b, b, mask, "f16", num_panels=7)
    ex = plan.export()
    ref = plan_ref.plan_from_mask(mask, plan.info()["group_rows"], plan.info()["num_panels"])
    for key in ("row_ptr", "col_idx", "panel_ptr"):
        assert np.array_equal(ex[key], ref[key]), key


@pytest.mark.parametrize("b", SMALL)
def test_small_sweep_shape_sampled_columns(b):
    """m = k = 8192, n = 1024, FP16, density 1/16: 64 seeded columns against the oracle."""
    c = Case(8192, 8192, 1024, b, 1 / 16, w="f16", seed=0)
    _, Y = c.run_static()
    cols = np.sort(np.random.default_rng(9).choice(1024, 64, replace=False))
    assert _err(c, Y, cols) <= 5e-3
    assert_elementwise(y_f64(Y, c)[:, cols], c.oracle(cols), c.abs_oracle(cols), c.k, "f16")
    assert torch.isfinite(Y).all().item()


@pytest.mark.parametrize("k_tail", [0, 1])  # k % b == 0 takes the one-workgroup encoder
@pytest.mark.parametrize("w", ["f16", "f32"])
@pytest.mark.parametrize("b", SMALL)
def test_small_dynamic_equals_static_bitwise(w, b, k_tail):
    c = Case(70 * b, 50 * b + k_tail, 300, b, 1 / 6, w=w, seed=40 + b)
    _, Ys = c.run_static()
    max_nnz = len(c.rows) + 9
    perm = np.random.default_rng(6).permutation(len(c.rows))
    pad = max_nnz - len(c.rows)
    r = dev(np.concatenate([c.rows[perm], np.zeros(pad, np.int32)]).astype(np.int32))
    col = dev(np.concatenate([c.cols[perm], np.zeros(pad, np.int32)]).astype(np.int32))
    v = dev(np.concatenate([c.vals_store[perm], np.zeros((pad, b, b), c.vals_store.dtype)]))
    nnz = torch.tensor([len(c.rows)], dtype=torch.int32, device="cuda")
    h = spmm.DynamicHandle(c.m, c.k, b, max_nnz, w)
    _, X, _ = c.device_inputs()
    Yd = c.new_Y()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, col, v, X, Yd, status, n=c.n)
    torch.cuda.synchronize()
    assert status.item() == 0
    assert torch.equal(Ys[:, : c.n], Yd[:, : c.n])
    assert _err(c, Yd) <= (1e-5 if w == "f32" else 5e-3)


@pytest.mark.parametrize("b", SMALL)
def test_small_dynamic_duplicates_summed(b):
    m, k, n = 33 * b, 21 * b, 130
    mb, kb = -(-m // b), -(-k // b)
    g = np.random.default_rng(b + 100)
    rows = g.integers(0, mb, 300).astype(np.int32)
    cols = g.integers(0, kb, 300).astype(np.int32)
    vals = synth.to_storage(synth.normal((300, b, b), 4), "f16")
    X = synth.to_storage(synth.normal((k, n), 5), "f16")
    h = spmm.DynamicHandle(m, k, b, 320, "f16", y="f32")
    Xd = torch.zeros((k, 136), dtype=torch.float16, device="cuda")
    Xd[:, :n] = dev(X)
    Y = torch.full((m, 136), float("nan"), dtype=torch.float32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pad = 20
    h.run(torch.tensor([300], dtype=torch.int32, device="cuda"),
          dev(np.concatenate([rows, np.zeros(pad, np.int32)])), dev(np.concatenate([cols, np.zeros(pad, np.int32)])),
          dev(np.concatenate([vals, np.zeros((pad, b, b), vals.dtype)])), Xd, Y, status, n=n)
    torch.cuda.synchronize()
    assert status.item() == 0
    ref = O.spmm_expand(m, k, b, rows, cols, synth.storage_to_f64(vals, "f16"), synth.storage_to_f64(X, "f16"))
    assert O.rel_fro(Y[:, :n].cpu().numpy().astype(np.float64), ref) <= 5e-3


@pytest.mark.parametrize("b,w,mbr,n", [(1, "f16", 300, 700), (1, "f32", 77, 300), (4, "f16", 90, 600), (8, "bf16", 61, 260),
                                       (4, "f16", 5, 200)])
def test_small_row_slices_equal_row_first_order_bitwise(b, w, mbr, n, monkeypatch):
    """The kernels without LDS order their units by 8, 4 or 2 slices of the
    row groups at large n; each unit is computed the same way as in the
    row-first order, so results are equal bit for bit, and integer data is
    exact against the oracle. Ragged m and n; fewer row groups than slices
    (mbr = 5)."""
    monkeypatch.setenv("SPMM_SMALL_LDS", "0")
    c = Case(mbr * b - (1 if b > 1 else 0), 53 * b + 3, n, b, 0.15, w=w, y="f32", seed=950 + b + mbr, integer=True)
    outs = []
    for sl in ("0", "8", "4", "2"):
        monkeypatch.setenv("SPMM_SMALL_SLICES", sl)
        plan, Y = c.run_static()
        assert np.array_equal(y_f64(Y, c), c.oracle()), sl
        assert torch.isnan(Y[:, c.n:]).all().item()
        outs.append(Y)
    for Y in outs[1:]:
        assert torch.equal(outs[0][:, : c.n], Y[:, : c.n])
