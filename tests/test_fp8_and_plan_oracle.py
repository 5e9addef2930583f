"""Pins of the FP8 decoder and the plan oracle (no GPU needed)."""
import numpy as np
import pytest
import torch

from oracle import fp8_ref, plan_ref
from paper_2303_16999_amd import synth


def test_e4m3fn_decode_table_matches_torch_for_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float32).numpy().astype(np.float64)
    ours = fp8_ref.decode_e4m3fn(codes)
    assert np.array_equal(np.isnan(ours), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(ours[fin], ref[fin])


def test_e4m3fn_known_values():
    d = fp8_ref.decode_e4m3fn
    assert d(0x7E) == 448.0 and d(0xFE) == -448.0
    assert d(0x38) == 1.0 and d(0x01) == 2.0 ** -9 and d(0x08) == 2.0 ** -6
    assert np.isnan(d(0x7F)) and np.isnan(d(0xFF))
    assert d(0x00) == 0.0 and np.signbit(d(0x80))


def test_quantizer_round_trip_and_saturation():
    vals = synth.scaled_block_values(64, 16, seed=3)
    codes, scales = synth.quantize_e4m3fn_blocks(vals)
    deq = fp8_ref.dequantize_blocks(codes, scales)
    v = vals.astype(np.float64)
    # amax of each block maps to exactly +-448 * s
    for z in range(vals.shape[0]):
        i = np.argmax(np.abs(v[z]))
        assert abs(fp8_ref.decode_e4m3fn(codes[z].reshape(-1)[i])) == 448.0
    # every value is within half a code spacing of its scaled value
    t = v / scales.astype(np.float64)[:, None, None]
    q = fp8_ref.decode_e4m3fn(codes)
    a = np.abs(q)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    ulp = 2.0 ** (e - 3)
    assert np.all(np.abs(q - t) <= ulp / 2 + 1e-12)
    # relative quantisation error of the whole set is a few percent at most
    err = np.linalg.norm(deq - v) / np.linalg.norm(v)
    assert err < 0.04
    # matches torch's own float8_e4m3fn rounding of t (RNE, values within range)
    tq = torch.from_numpy(t.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # torch rounds the float32 copy of t; compare only where t is exactly representable in float32
    exact = t.astype(np.float32).astype(np.float64) == t
    assert np.array_equal(tq[exact], codes[exact])


def test_zero_block_scale_is_one():
    codes, scales = synth.quantize_e4m3fn_blocks(np.zeros((2, 4, 4), np.float32))
    assert np.all(scales == 1.0) and not codes.any()


def _check_plan_properties(M, R, P, pl):
    mb, kb = M.shape
    row_ptr, col_idx, panel_ptr, order = (np.asarray(pl[x]) for x in ("row_ptr", "col_idx", "panel_ptr", "order"))
    assert row_ptr[0] == 0 and np.all(np.diff(row_ptr) == M.sum(axis=1))
    for r in range(mb):
        seg = col_idx[row_ptr[r]:row_ptr[r + 1]]
        assert np.array_equal(seg, np.flatnonzero(M[r]))
    G = -(-mb // R)
    assert panel_ptr[0] == 0 and panel_ptr[-1] == G and np.all(np.diff(panel_ptr) >= 0)
    assert sorted(order.tolist()) == list(range(int(M.sum())))


@pytest.mark.parametrize("R,P", [(1, 1), (2, 3), (4, 2), (3, 7), (8, 1)])
def test_plan_numpy_equals_loops(R, P):
    g = np.random.default_rng(R * 10 + P)
    for trial in range(5):
        mb, kb = int(g.integers(1, 20)), int(g.integers(1, 20))
        M = (g.random((mb, kb)) < [0.0, 1.0, 0.2, 0.5, 0.05][trial]).astype(np.uint8)
        a = plan_ref.plan_from_mask(M, R, P)
        b = plan_ref.plan_loops(M, R, P)
        for key in ("row_ptr", "col_idx", "panel_ptr", "order", "group_cost_prefix"):
            assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key
        _check_plan_properties(M, R, P, a)


def test_plan_panels_balance_cost():
    M = synth.block_mask(512, 512, 1 / 16, seed=1)
    R, P = 8, 16
    pl = plan_ref.plan_from_mask(M, R, P)
    C = pl["group_cost_prefix"]
    pp = pl["panel_ptr"]
    costs = C[pp[1:]] - C[pp[:-1]]
    G = len(C) - 1
    wmax = np.max(np.diff(C))
    # each panel is within one group's cost of the ideal share
    assert np.all(np.abs(costs - C[-1] / P) <= wmax)
    assert pp[-1] == G


def test_dynamic_plan_is_canonical_and_order_independent():
    g = np.random.default_rng(4)
    mb, kb, R, P = 9, 7, 4, 2
    rows = g.integers(0, mb, size=30)
    cols = g.integers(0, kb, size=30)  # duplicates likely
    a = plan_ref.plan_from_coo(mb, kb, rows, cols, R, P)
    perm = g.permutation(30)
    b = plan_ref.plan_from_coo(mb, kb, rows[perm], cols[perm], R, P)
    assert np.array_equal(a["row_ptr"], b["row_ptr"]) and np.array_equal(a["col_idx"], b["col_idx"])
    # the CSR list is sorted by (row, col) and duplicates keep input order
    keys = [(int(rows[s]), int(cols[s]), int(s)) for s in a["src"]]
    assert keys == sorted(keys)
    # without duplicates the COO plan equals the mask plan, with order mapped through src
    flat = np.unique(rows * kb + cols)
    r2, c2 = flat // kb, flat % kb
    p2 = g.permutation(len(flat))
    dyn = plan_ref.plan_from_coo(mb, kb, r2[p2], c2[p2], R, P)
    M = np.zeros((mb, kb), np.uint8)
    M[r2, c2] = 1
    st = plan_ref.plan_from_mask(M, R, P)
    for key in ("row_ptr", "col_idx", "panel_ptr"):
        assert np.array_equal(dyn[key], st[key])
    with pytest.raises(IndexError):
        plan_ref.plan_from_coo(mb, kb, [mb], [0], R, P)


def test_mask_generator_exact_count_and_seed_stability():
    M1 = synth.block_mask(64, 48, 1 / 16, seed=5)
    M2 = synth.block_mask(64, 48, 1 / 16, seed=5)
    assert M1.sum() == round(64 * 48 / 16) and np.array_equal(M1, M2)
    assert not np.array_equal(M1, synth.block_mask(64, 48, 1 / 16, seed=6))


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38], np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(synth.to_bf16_bits(x), ref)
