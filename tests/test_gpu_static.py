"""GPU parity of the static path against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from oracle import plan_ref
from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import assert_elementwise, TOL, Case, dev, round_like, y_f64

pytestmark = pytest.mark.gpu


def _check(case, Y, cols=None, tol=None):
    ref = case.oracle(cols)
    got = y_f64(Y, case) if cols is None else y_f64(Y, case)[:, cols]
    err = O.rel_fro(got, ref)
    assert np.all(np.isfinite(got)), "non-finite output"
    assert err <= (tol or TOL[case.y if case.y != "f32" or case.x == "f32" else case.x]), err
    return err


def test_config1_fp32_small_static():
    """W 1024x1024, b=16, d=1/16, FP32 N(0,1); X 1024x64 FP32."""
    c = Case(1024, 1024, 64, 16, 1 / 16, w="f32", seed=0)
    _, Y = c.run_static()
    assert _check(c, Y, tol=1e-5) <= 1e-5


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "bf16"), ("f16", "f32"), ("bf16", "f32"), ("f32", "f32")])
@pytest.mark.parametrize("b", [16, 32])
def test_ragged_shapes_all_dtypes(w, y, b):
    # several row groups, chunks and n-tiles, with partial edge blocks and an n tail
    m, k, n = 7 * b + 5, 13 * b + 3, 300
    c = Case(m, k, n, b, 0.3, w=w, y=y, seed=3)
    _, Y = c.run_static()
    _check(c, Y, tol=1e-5 if w == "f32" else 5e-3)


@pytest.mark.parametrize("x,y", [("f16", "f16"), ("bf16", "bf16"), ("bf16", "f32"), ("f16", "f32")])
@pytest.mark.parametrize("b", [16, 32])
def test_fp8_block_scales(x, y, b):
    c = Case(9 * b, 11 * b + 7, 200, b, 0.35, w="fp8", x=x, y=y, seed=5, scaled=True)
    _, Y = c.run_static()
    _check(c, Y, tol=5e-3)


@pytest.mark.parametrize("w", ["f16", "bf16", "f32", "fp8"])
@pytest.mark.parametrize("b", [16, 32])
def test_integer_data_bit_exact(w, b):
    # entries in {-2..2}: every partial sum is an exact small integer, so the
    # device result must equal the oracle bit for bit after rounding to Y
    c = Case(6 * b, 10 * b, 130, b, 0.25, w=w, seed=7, integer=True)
    _, Y = c.run_static()
    got = y_f64(Y, c)
    ref = c.oracle()
    assert np.abs(ref).max() <= 256
    assert np.array_equal(got, round_like(ref, c.y))


@pytest.mark.parametrize("w", ["f16", "bf16", "f32"])
def test_identity_block_permutation_bit_exact(w):
    b, nb, n = 16, 24, 96
    perm = np.random.default_rng(1).permutation(nb)
    mask = np.zeros((nb, nb), np.uint8)
    mask[np.arange(nb), perm] = 1
    c = Case(nb * b, nb * b, n, b, 0.0, w=w, seed=2, mask=mask)
    eye = np.stack([np.eye(b, dtype=np.float32)] * nb)
    from paper_2303_16999_amd import synth
    c.vals_store = synth.to_storage(eye, w)
    c.vals64 = synth.storage_to_f64(c.vals_store, w)
    _, Y = c.run_static()
    got = y_f64(Y, c)
    expect = np.concatenate([c.X64[col * b:(col + 1) * b] for col in perm])
    assert np.array_equal(got, expect)


def test_density_zero_overwrites_nan():
    c = Case(100, 70, 50, 16, 0.0, w="f16")
    _, Y = c.run_static()
    assert torch.all(Y[:, :50] == 0).item()
    assert torch.isnan(Y[:, 50:]).all().item() if Y.shape[1] > 50 else True


def test_empty_rows_and_untouched_columns_beyond_n():
    c = Case(160, 96, 40, 16, 0.5, w="f16", seed=4, ldy=64)
    mask = c.mask.copy()
    mask[3] = 0
    c = Case(160, 96, 40, 16, 0.5, w="f16", seed=4, ldy=64, mask=mask)
    _, Y = c.run_static()
    _check(c, Y)
    assert torch.all(Y[48:64, :40] == 0).item()
    assert torch.isnan(Y[:, 40:]).all().item()  # columns in [n, ldy) are never written


def test_deterministic_and_repeatable():
    c = Case(512, 640, 384, 16, 1 / 8, w="f16", seed=9)
    plan, Y1 = c.run_static()
    vals, X, scales = c.device_inputs()
    Y2 = c.new_Y()
    plan.run(X, Y2, n=c.n)
    torch.cuda.synchronize()
    assert torch.equal(Y1[:, : c.n], Y2[:, : c.n])


@pytest.mark.parametrize("P", [1, 2, 5])
def test_panels_walk_several_groups(P):
    c = Case(40 * 16, 24 * 16, 200, 16, 0.2, w="bf16", seed=11)
    plan, Y = c.run_static(group_rows=8, num_panels=P)
    _check(c, Y)
    ex = plan.export()
    ref = plan_ref.plan_from_mask(c.mask, 8, P)
    for key in ("row_ptr", "col_idx", "panel_ptr"):
        assert np.array_equal(ex[key], ref[key]), key


@pytest.mark.parametrize("b,mb,kb,d,gr,P", [(16, 64, 64, 1 / 16, 32, 2), (16, 33, 70, 0.4, 8, 5),
                                            (32, 17, 9, 0.5, 8, 3), (32, 64, 40, 0.1, 16, 4),
                                            (16, 512, 512, 1 / 16, 32, 16), (16, 1, 1, 1.0, 8, 1)])
def test_gpu_plan_bit_exact_vs_oracle(b, mb, kb, d, gr, P):
    from paper_2303_16999_amd import synth
    mask = synth.block_mask(mb, kb, d, seed=mb + kb)
    plan = spmm.StaticPlan(mb * b, kb * b, b, mask, "f16", group_rows=gr, num_panels=P)
    ex = plan.export()
    ref = plan_ref.plan_from_mask(mask, gr, P)
    for key in ("row_ptr", "col_idx", "panel_ptr"):
        assert np.array_equal(ex[key], ref[key]), key

def test_headline_shape_sampled_columns():
    """m=k=8192, n=4096, b=16, d=1/16, FP16: 128 seeded columns against the
    oracle (exact by column separability), relative Frobenius error and every
    element within its rounding bound; the rest for finiteness."""
    c = Case(8192, 8192, 4096, 16, 1 / 16, w="f16", seed=0)
    _, Y = c.run_static()
    cols = np.sort(np.random.default_rng(123).choice(4096, 128, replace=False))
    got, ref = y_f64(Y, c)[:, cols], c.oracle(cols)
    err = O.rel_fro(got, ref)
    assert err <= 5e-3, err
    assert_elementwise(got, ref, c.abs_oracle(cols), c.k, "f16")
    assert torch.isfinite(Y).all().item()


def test_default_plan_holds_one_copy_of_the_values():
    # b = 16, FP16, the headline pattern: values once, plus int32 indices
    m = k = 8192
    b = 16
    mask = synth.block_mask(m // b, k // b, 1 / 16, 0)
    nnzb = int(mask.sum())
    vals = torch.zeros((nnzb, b, b), dtype=torch.float16, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan = spmm.StaticPlan(m, k, b, mask, "f16")
    plan.set_values(vals)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    dev_bytes, val_bytes = plan.memory()
    assert val_bytes == nnzb * b * b * 2
    # indices: col_idx and the in-group order (4 + 4 bytes per block), the
    # tiled SDDMM's entry list (8 bytes per block), row pointers, panels,
    # scratch and the task lists, 16 B per tiled task (at most one per
    # 256 x 256 tile plus one per 24 blocks): under 64 KiB + 21 B/block + 16 B/tile
    tiles = (m // 256) * (k // 256)
    assert val_bytes < dev_bytes <= val_bytes + 21 * nnzb + 16 * tiles + 64 * 1024
    # what the device lost to the plan: one copy, never two (allocation rounding aside)
    assert free0 - free1 < 1.5 * val_bytes + 4 * 2**20
    plan.close()


@pytest.mark.parametrize("b,mb,n,ns", [(16, 37, 1000, 8), (16, 37, 300, 4), (16, 5, 700, 2), (32, 23, 520, 8),
                                       (16, 61, 100, 8)])
def test_row_slices_equal_row_first_order_bitwise(b, mb, n, ns, monkeypatch):
    """Light units by eighths of the block rows (the default from n = 16384)
    cover the same (row group, column step) units as the row-first order,
    each computed the same way: results equal bit for bit, integer data
    exact against the oracle. Ragged m and n; fewer row groups than eight
    (mb = 5); one tile (n = 100 with ns = 8: four rows per unit)."""
    c = Case(mb * b - 3, 41 * b - 5, n, b, 0.2, w="f16", y="f32", seed=900 + mb, integer=True)
    outs = []
    for sl in ("0", "1"):
        monkeypatch.setenv("SPMM_ROW_SLICES", sl)
        plan = spmm.StaticPlan(c.m, c.k, b, c.mask, "f16", y="f32", variant=ns + 256)
        vals, X, _ = c.device_inputs()
        plan.set_values(vals)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        assert np.array_equal(y_f64(Y, c), c.oracle()), sl
        assert torch.isnan(Y[:, c.n:]).all().item()
        outs.append(Y)
    assert torch.equal(outs[0][:, : c.n], outs[1][:, : c.n])


def test_slice_orders_at_large_n_all_paths(monkeypatch):
    """At the n where units go by row slices (row kernel from n = 16384, the
    small-block kernels without LDS from n = 8192 or 16384): the static plan
    is exact on integer data and equal bit for bit to the row-first order; a
    grouped launch holding such a problem equals its single launch; a dynamic
    call equals the static plan."""
    monkeypatch.setenv("SPMM_SMALL_LDS", "0")
    # row kernel, n = 16384
    c = Case(37 * 16 - 3, 25 * 16, 16384, 16, 0.2, w="f16", y="f32", seed=960, integer=True)
    outs = []
    for sl in ("", "0"):
        if sl:
            monkeypatch.setenv("SPMM_ROW_SLICES", sl)
        plan, Y = c.run_static()
        assert np.array_equal(y_f64(Y, c), c.oracle()), sl
        outs.append((plan, Y))
    monkeypatch.delenv("SPMM_ROW_SLICES", raising=False)
    assert torch.equal(outs[0][1][:, : c.n], outs[1][1][:, : c.n])
    # a grouped launch of that plan (n = 16384) and a small problem
    c2 = Case(37 * 16 - 3, 25 * 16, 300, 16, 0.2, w="f16", y="f32", seed=961, integer=True)
    p2, Y2 = c2.run_static()
    _, X1, _ = c.device_inputs()
    _, X2, _ = c2.device_inputs()
    G1, G2 = c.new_Y(), c2.new_Y()
    spmm.Group(4).run([outs[0][0], p2], [X1, X2], [G1, G2], ns=[c.n, c2.n])
    torch.cuda.synchronize()
    assert torch.equal(G1[:, : c.n], outs[0][1][:, : c.n])
    assert torch.equal(G2[:, : c2.n], Y2[:, : c2.n])
    # small-block kernels without LDS at their slice thresholds
    for b, n in ((1, 16384), (4, 8192), (8, 8192)):
        cs = Case(29 * b + 1, 31 * b, n, b, 0.2, w="f16", y="f32", seed=962 + b, integer=True)
        res = []
        for sl in ("", "0"):
            if sl:
                monkeypatch.setenv("SPMM_SMALL_SLICES", sl)
            _, Ys = cs.run_static()
            assert np.array_equal(y_f64(Ys, cs), cs.oracle()), (b, sl)
            res.append(Ys)
        monkeypatch.delenv("SPMM_SMALL_SLICES", raising=False)
        assert torch.equal(res[0][:, : cs.n], res[1][:, : cs.n]), b
    # a dynamic call at b = 4, n = 8192 against the static plan (both sliced)
    cd = Case(29 * 4 + 1, 31 * 4, 8192, 4, 0.2, w="f16", seed=970)
    _, Ys = cd.run_static()
    max_nnz = len(cd.rows) + 3
    pad = max_nnz - len(cd.rows)
    perm = np.random.default_rng(9).permutation(len(cd.rows))
    r = dev(np.concatenate([cd.rows[perm], np.zeros(pad, np.int32)]).astype(np.int32))
    col = dev(np.concatenate([cd.cols[perm], np.zeros(pad, np.int32)]).astype(np.int32))
    v = dev(np.concatenate([cd.vals_store[perm], np.zeros((pad, 4, 4), cd.vals_store.dtype)]))
    nnz = torch.tensor([len(cd.rows)], dtype=torch.int32, device="cuda")
    h = spmm.DynamicHandle(cd.m, cd.k, 4, max_nnz, "f16")
    _, X, _ = cd.device_inputs()
    Yd = cd.new_Y()
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, col, v, X, Yd, st, n=cd.n)
    torch.cuda.synchronize()
    assert st.item() == 0
    assert torch.equal(Ys[:, : cd.n], Yd[:, : cd.n])


def test_large_n_full_size_sampled_columns():
    """m = k = 8192, n = 16384, b = 16, d = 1/16, FP16 (units by row slices):
    128 seeded columns against the oracle (exact by column separability),
    every element within its rounding bound; the rest for finiteness."""
    c = Case(8192, 8192, 16384, 16, 1 / 16, w="f16", seed=3)
    _, Y = c.run_static()
    cols = np.sort(np.random.default_rng(321).choice(16384, 128, replace=False))
    got, ref = y_f64(Y, c)[:, cols], c.oracle(cols)
    assert O.rel_fro(got, ref) <= 5e-3
    assert_elementwise(got, ref, c.abs_oracle(cols), c.k, "f16")
    assert torch.isfinite(Y[:, : c.n]).all().item()


def test_b1_lds_full_size_sampled_rows_and_columns():
    """m = k = 8192, n = 4096, b = 1, d = 1/8, FP16 (the LDS-staged kernel by
    the rule): 64 seeded rows x 128 seeded columns against the oracle given
    only those rows' entries (exact by row and column separability), every
    element within its rounding bound."""
    c = Case(8192, 8192, 4096, 1, 1 / 8, w="f16", seed=4)
    _, Y = c.run_static()
    g = np.random.default_rng(654)
    rs = np.sort(g.choice(8192, 64, replace=False))
    cs = np.sort(g.choice(4096, 128, replace=False))
    sel = np.isin(c.rows, rs)
    rows, cols, vals = c.rows[sel], c.cols[sel], c.vals64[sel]
    ref = O.spmm_blockwise_columns(c.m, c.k, 1, rows, cols, vals, c.X64, cs)[rs]
    bound = O.spmm_blockwise_columns(c.m, c.k, 1, rows, cols, np.abs(vals), np.abs(c.X64), cs)[rs]
    got = y_f64(Y, c)[rs][:, cs]
    assert O.rel_fro(got, ref) <= 5e-3
    assert_elementwise(got, ref, bound, c.k, "f16")
    assert torch.isfinite(Y[:, : c.n]).all().item()


@pytest.mark.parametrize("b,n", [(4, 16384), (8, 8192)])
def test_small_blocks_large_n_full_size_sampled_columns(b, n):
    """m = k = 8192, d = 1/16, FP16 at large n: b = 4 at n = 16384 (the
    LDS-staged kernel by the rule) and b = 8 at n = 8192 (the kernel without
    LDS, units by row slices): 64 seeded columns against the oracle, every
    element within its rounding bound."""
    c = Case(8192, 8192, n, b, 1 / 16, w="f16", seed=5 + b)
    _, Y = c.run_static()
    cols = np.sort(np.random.default_rng(77 + b).choice(n, 64, replace=False))
    got, ref = y_f64(Y, c)[:, cols], c.oracle(cols)
    assert O.rel_fro(got, ref) <= 5e-3
    assert_elementwise(got, ref, c.abs_oracle(cols), c.k, "f16")
    assert torch.isfinite(Y[:, : c.n]).all().item()
