"""GPU parity of the dynamic path: oracle, static equivalence, status words."""
import numpy as np
import pytest
import torch

from oracle import plan_ref
from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import assert_elementwise, Case, dev, y_f64

pytestmark = pytest.mark.gpu


def _dyn_inputs(rows, cols, vals_store, max_nnz, b):
    pad = max_nnz - len(rows)
    r = np.concatenate([rows, np.zeros(pad, np.int32)]).astype(np.int32)
    c = np.concatenate([cols, np.zeros(pad, np.int32)]).astype(np.int32)
    v = np.concatenate([vals_store, np.zeros((pad,) + vals_store.shape[1:], vals_store.dtype)])
    return dev(r), dev(c), dev(v), torch.tensor([len(rows)], dtype=torch.int32, device="cuda")


def test_dynamic_matches_oracle_and_static_bitwise():
    # the static plan by the rule a dynamic call follows (tile width 8 for n =
    # 256, kernel form by rule), whatever a tuned table holds
    c = Case(48 * 16, 40 * 16, 256, 16, 1 / 8, w="f16", seed=21)
    plan = spmm.StaticPlan(c.m, c.k, 16, c.mask, "f16", group_rows=8, variant=8)
    vals, X0, _ = c.device_inputs()
    plan.set_values(vals)
    Ys = c.new_Y()
    plan.run(X0, Ys, n=c.n)
    torch.cuda.synchronize()
    max_nnz = len(c.rows) + 17
    perm = np.random.default_rng(5).permutation(len(c.rows))  # COO in random order
    r, col, v, nnz = _dyn_inputs(c.rows[perm], c.cols[perm], c.vals_store[perm], max_nnz, 16)
    h = spmm.DynamicHandle(c.m, c.k, 16, max_nnz, "f16", group_rows=8)
    _, X, _ = c.device_inputs()
    Yd = c.new_Y()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, col, v, X, Yd, status, n=c.n)
    torch.cuda.synchronize()
    assert status.item() == 0
    assert torch.equal(Ys[:, : c.n], Yd[:, : c.n])
    assert O.rel_fro(y_f64(Yd, c), c.oracle()) <= 5e-3
    ex = h.export()
    ref = plan_ref.plan_from_coo(h.mb, h.kb, c.rows[perm], c.cols[perm], 8, h.info()["num_panels"])
    for key in ("row_ptr", "col_idx", "panel_ptr"):
        assert np.array_equal(ex[key], ref[key]), key
    assert np.array_equal(ex["src"], ref["src"])


def test_dynamic_duplicates_summed_and_ragged():
    b, m, k, n = 16, 150, 90, 70
    mb, kb = -(-m // b), -(-k // b)
    g = np.random.default_rng(3)
    rows = g.integers(0, mb, 40).astype(np.int32)
    cols = g.integers(0, kb, 40).astype(np.int32)
    vals = synth.to_storage(synth.normal((40, b, b), 4), "bf16")
    X = synth.to_storage(synth.normal((k, n), 5), "bf16")
    r, c, v, nnz = _dyn_inputs(rows, cols, vals, 64, b)
    h = spmm.DynamicHandle(m, k, b, 64, "bf16", y="f32")
    Xd = torch.zeros((k, 72), dtype=torch.bfloat16, device="cuda")
    Xd[:, :n] = dev(X)
    Y = torch.full((m, 72), float("nan"), dtype=torch.float32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, c, v, Xd, Y, status, n=n)
    torch.cuda.synchronize()
    assert status.item() == 0
    ref = O.spmm_expand(m, k, b, rows, cols, synth.storage_to_f64(vals, "bf16"), synth.storage_to_f64(X, "bf16"))
    assert O.rel_fro(Y[:, :n].cpu().numpy(), ref) <= 5e-3


def test_dynamic_capacity_and_bad_index_leave_y_untouched():
    b, m, k, n = 16, 64, 64, 32
    h = spmm.DynamicHandle(m, k, b, 8, "f16")
    X = torch.ones((k, n), dtype=torch.float16, device="cuda")
    v = torch.ones((8, b, b), dtype=torch.float16, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for rows, cols, nnz, want in [([0] * 8, [0] * 8, 9, spmm.ERR_CAPACITY), ([0] * 8, [0] * 8, -1, spmm.ERR_CAPACITY),
                                  ([0, 4] + [0] * 6, [0, 1] + [0] * 6, 2, spmm.ERR_BAD_INDEX),
                                  ([0, 1] + [0] * 6, [0, -1] + [0] * 6, 2, spmm.ERR_BAD_INDEX)]:
        Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
        r = torch.tensor(rows, dtype=torch.int32, device="cuda")
        c = torch.tensor(cols, dtype=torch.int32, device="cuda")
        nz = torch.tensor([nnz], dtype=torch.int32, device="cuda")
        h.run(nz, r, c, v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == want
        assert torch.all(Y == 7.0).item()
    # the handle recovers on the next valid call
    nz = torch.tensor([1], dtype=torch.int32, device="cuda")
    r = torch.zeros(8, dtype=torch.int32, device="cuda")
    Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
    h.run(nz, r, r, v, X, Y, status)
    torch.cuda.synchronize()
    assert status.item() == 0
    assert torch.all(Y[:16] == 16.0).item() and torch.all(Y[16:] == 0).item()


@pytest.mark.parametrize("w", ["f16", "fp8"])
def test_dynamic_call_stream_config3_shape(w):
    """m=k=4096, n=512, b=16, max density 1/8: a few calls with fresh patterns."""
    b, m, k, n = 16, 4096, 4096, 512
    mb = kb = 256
    max_nnz = mb * kb // 8
    h = spmm.DynamicHandle(m, k, b, max_nnz, w, x="f16")
    X_store = synth.to_storage(synth.normal((k, n), 2), "f16")
    X = dev(X_store)
    X64 = synth.storage_to_f64(X_store, "f16")
    cols_s = np.sort(np.random.default_rng(0).choice(n, 64, replace=False))
    for i in range(3):
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=3 + i, dtype="f16")
        scales = None
        if w == "fp8":
            codes, sc = synth.quantize_e4m3fn_blocks(synth.storage_to_f64(vals, "f16").astype(np.float32))
            from oracle import fp8_ref
            v64 = fp8_ref.dequantize_blocks(codes, sc)
            vals_dev = dev(np.concatenate([codes, np.zeros((max_nnz - len(rows), b, b), np.uint8)]))
            scales = dev(np.concatenate([sc, np.ones(max_nnz - len(rows), np.float32)]))
        else:
            v64 = synth.storage_to_f64(vals, "f16")
            vals_dev = None
        r, c, v, nnz = _dyn_inputs(rows, cols, vals if w != "fp8" else np.zeros((len(rows), b, b), np.float16),
                                   max_nnz, b)
        if vals_dev is not None:
            v = vals_dev
        Y = torch.full((m, n), float("nan"), dtype=torch.float16, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, X, Y, status, scales=scales)
        torch.cuda.synchronize()
        assert status.item() == 0
        ref = O.spmm_blockwise_columns(m, k, b, rows, cols, v64, X64, cols_s)
        got = Y.cpu().numpy().astype(np.float64)[:, cols_s]
        assert O.rel_fro(got, ref) <= 5e-3
        A = O.spmm_blockwise_columns(m, k, b, rows, cols, np.abs(v64), np.abs(X64), cols_s)
        assert_elementwise(got, ref, A, 2 * k if w == "fp8" else k, "f16")


@pytest.mark.parametrize("w,b", [("f16", 16), ("fp8", 16), ("bf16", 32)])
def test_one_workgroup_encoder_equals_multi_kernel_encoder(w, b, monkeypatch):
    """Both dynamic encoders give the same plan (and the oracle's) and the same Y bit for bit."""
    m = k = 64 * b
    mb = kb = 64
    max_nnz = mb * kb // 8
    x = "bf16" if w == "fp8" else None
    h = spmm.DynamicHandle(m, k, b, max_nnz, w, x=x, group_rows=8 if b == 16 else 0, num_panels=5)
    rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=17, dtype="f16")
    scales = None
    if w == "fp8":
        codes, sc = synth.quantize_e4m3fn_blocks(synth.storage_to_f64(vals, "f16").astype(np.float32))
        pad = max_nnz - len(rows)
        v = dev(np.concatenate([codes, np.zeros((pad, b, b), np.uint8)]))
        scales = dev(np.concatenate([sc, np.ones(pad, np.float32)]))
        r, c, _, nnz = _dyn_inputs(rows, cols, np.zeros((len(rows), b, b), np.float16), max_nnz, b)
    else:
        vals = synth.to_storage(synth.storage_to_f64(vals, "f16"), w)
        r, c, v, nnz = _dyn_inputs(rows, cols, vals, max_nnz, b)
    X = dev(synth.to_storage(synth.normal((k, 192), 3), x or w))
    outs, exports = [], []
    for builder in (None, "one", "multi"):
        if builder:
            monkeypatch.setenv("SPMM_DYN_BUILDER", builder)
        else:
            monkeypatch.delenv("SPMM_DYN_BUILDER", raising=False)
        Y = torch.full((m, 192), float("nan"), dtype=X.dtype, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, X, Y, status, scales=scales)
        torch.cuda.synchronize()
        assert status.item() == 0
        outs.append(Y)
        exports.append(h.export())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    ref = plan_ref.plan_from_coo(mb, kb, rows, cols, h.info()["group_rows"], h.info()["num_panels"])
    for ex in exports:
        for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
            assert np.array_equal(ex[key], ref[key]), key


@pytest.mark.parametrize("case", ["config3", "skewed", "ragged", "empty", "wide"])
def test_row_range_encoder_equals_one_workgroup_encoder(case, monkeypatch):
    """The row-range encoder (one workgroup per range of block rows) gives the
    oracle's plan and the one-workgroup encoder's Y bit for bit: the dynamic
    benchmark's grid, every entry in the first rows with repeated pairs (one
    workgroup ranks them all), a block-row count its ranges do not divide,
    an empty call, and more block columns than the bitmap form takes."""
    b, n = 16, 80
    g = np.random.default_rng(31)
    if case == "config3":
        mb, kb, max_nnz = 256, 256, 8192
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=32)
    elif case == "skewed":
        mb, kb, max_nnz = 300, 64, 3000
        rows = g.integers(0, 3, 2900).astype(np.int32)
        cols = g.integers(0, kb, 2900).astype(np.int32)
        vals = synth.to_storage(synth.normal((2900, b, b), 33), "f16")
    elif case == "ragged":
        mb, kb, max_nnz = 301, 50, 4000
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=34)
    elif case == "empty":
        mb, kb, max_nnz = 40, 30, 100
        rows, cols = np.zeros(0, np.int32), np.zeros(0, np.int32)
        vals = np.zeros((0, b, b), np.float16)
    else:
        mb, kb, max_nnz = 8, 1100, 2000
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=35)
    m, k = mb * b, kb * b
    h = spmm.DynamicHandle(m, k, b, max_nnz, "f16", num_panels=5)
    r, c, v, nnz = _dyn_inputs(rows, cols, vals, max_nnz, b)
    X = dev(synth.to_storage(synth.normal((k, n), 36), "f16"))
    outs, exports = [], []
    for builder in ("rows", "one"):
        monkeypatch.setenv("SPMM_DYN_BUILDER", builder)
        Y = torch.full((m, n), float("nan"), dtype=torch.float16, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == 0
        outs.append(Y)
        exports.append(h.export())
    assert torch.equal(outs[0], outs[1])
    ref = plan_ref.plan_from_coo(mb, kb, rows, cols, h.info()["group_rows"], h.info()["num_panels"])
    for ex in exports:
        assert ex["nnzb"] == len(rows)
        for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
            assert np.array_equal(ex[key], ref[key]), key
    if case == "empty":
        assert torch.all(outs[0] == 0).item()


def test_row_range_encoder_status_words(monkeypatch):
    monkeypatch.setenv("SPMM_DYN_BUILDER", "rows")
    b, m, k, n = 16, 64 * 16, 64 * 16, 32
    h = spmm.DynamicHandle(m, k, b, 100, "f16")
    X = torch.ones((k, n), dtype=torch.float16, device="cuda")
    v = torch.ones((100, b, b), dtype=torch.float16, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    base_r = list(range(50)) + [0] * 50
    for rows, cols, nnz, want in [(base_r, [1] * 100, 101, spmm.ERR_CAPACITY),
                                  (base_r[:49] + [64] + [0] * 50, [1] * 100, 50, spmm.ERR_BAD_INDEX),
                                  (base_r, [1] * 30 + [70] + [1] * 69, 50, spmm.ERR_BAD_INDEX)]:
        Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
        r = torch.tensor(rows, dtype=torch.int32, device="cuda")
        c = torch.tensor(cols, dtype=torch.int32, device="cuda")
        nz = torch.tensor([nnz], dtype=torch.int32, device="cuda")
        h.run(nz, r, c, v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == want
        assert torch.all(Y == 7.0).item()
    nz = torch.tensor([50], dtype=torch.int32, device="cuda")
    r = torch.tensor(base_r, dtype=torch.int32, device="cuda")
    c = torch.ones(100, dtype=torch.int32, device="cuda")
    Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
    h.run(nz, r, c, v, X, Y, status)
    torch.cuda.synchronize()
    assert status.item() == 0
    assert torch.all(Y[: 50 * b] == 16.0).item() and torch.all(Y[50 * b:] == 0).item()


@pytest.mark.parametrize("b", [16, 32])
@pytest.mark.parametrize("ragged", [False, True])
def test_dynamic_fp32_matches_static_and_oracle(b, ragged):
    # FP32 dynamic calls run the row-wise FP32 kernel: bitwise equal to the static plan of the same
    # pattern; a k that b does not divide goes through the copying encoder
    m, k = 37 * b + (5 if ragged else 0), 29 * b + (b // 2 if ragged else 0)
    c = Case(m, k, 150, b, 1 / 6, w="f32", seed=300 + b)
    plan, Ys = c.run_static()
    max_nnz = len(c.rows) + 9
    perm = np.random.default_rng(6).permutation(len(c.rows))
    r, col, v, nnz = _dyn_inputs(c.rows[perm], c.cols[perm], c.vals_store[perm], max_nnz, b)
    h = spmm.DynamicHandle(c.m, c.k, b, max_nnz, "f32")
    _, X, _ = c.device_inputs()
    Yd = c.new_Y()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, col, v, X, Yd, status, n=c.n)
    torch.cuda.synchronize()
    assert status.item() == 0
    assert torch.equal(Ys[:, : c.n], Yd[:, : c.n])
    assert O.rel_fro(y_f64(Yd, c), c.oracle()) <= 1e-5


def test_dynamic_fp32_bad_index_leaves_y_untouched():
    b, m, k = 16, 160, 160
    h = spmm.DynamicHandle(m, k, b, 8, "f32")
    r = torch.tensor([0, 1, 99, 0, 0, 0, 0, 0], dtype=torch.int32, device="cuda")
    c = torch.zeros(8, dtype=torch.int32, device="cuda")
    v = torch.ones((8, b, b), dtype=torch.float32, device="cuda")
    nnz = torch.tensor([3], dtype=torch.int32, device="cuda")
    X = torch.ones((k, 16), dtype=torch.float32, device="cuda")
    Y = torch.full((m, 16), 7.0, dtype=torch.float32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, c, v, X, Y, status)
    torch.cuda.synchronize()
    assert status.item() == spmm.ERR_BAD_INDEX
    assert bool((Y == 7.0).all())


@pytest.mark.parametrize("case", ["config3", "chunked", "wide", "repeats"])
def test_bitmap_rank_equals_pairwise_rank(case, monkeypatch):
    """The one-workgroup encoder's column-bitmap ranking and its pairwise ranking
    give the oracle's plan and the same Y bit for bit: at the dynamic benchmark's
    grid (256 x 256 blocks), above the entries one pass keeps in registers
    (8800 > 8192), past the bitmap's 1024-column limit (the pairwise path then
    runs in both), and with repeated (row, column) pairs (which switch the
    bitmap form to the pairwise ranking inside the kernel)."""
    b, n = 16, 96
    g = np.random.default_rng(91)
    if case == "config3":
        mb, kb, max_nnz = 256, 256, 8192
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=92)
    elif case == "chunked":
        mb, kb, max_nnz = 16, 600, 8800
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=93, lo_frac=1.0)
    elif case == "wide":
        mb, kb, max_nnz = 8, 1100, 2000
        rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=94)
    else:
        mb, kb, max_nnz = 40, 40, 600
        rows = g.integers(0, mb, 500).astype(np.int32)
        cols = g.integers(0, kb, 500).astype(np.int32)
        rows[100:120], cols[100:120] = rows[:20], cols[:20]  # certain repeats
        vals = synth.to_storage(synth.normal((500, b, b), 95), "f16")
    assert len(rows) <= max_nnz
    m, k = mb * b, kb * b
    h = spmm.DynamicHandle(m, k, b, max_nnz, "f16", num_panels=7)
    r, c, v, nnz = _dyn_inputs(rows, cols, vals, max_nnz, b)
    X = dev(synth.to_storage(synth.normal((k, n), 96), "f16"))
    outs, exports = [], []
    monkeypatch.setenv("SPMM_DYN_BUILDER", "one")
    for rank in (None, "pairwise"):
        if rank:
            monkeypatch.setenv("SPMM_DYN_RANK", rank)
        else:
            monkeypatch.delenv("SPMM_DYN_RANK", raising=False)
        Y = torch.full((m, n), float("nan"), dtype=torch.float16, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == 0
        outs.append(Y)
        exports.append(h.export())
    assert torch.equal(outs[0], outs[1])
    ref = plan_ref.plan_from_coo(mb, kb, rows, cols, h.info()["group_rows"], h.info()["num_panels"])
    for ex in exports:
        for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
            assert np.array_equal(ex[key], ref[key]), key
    if case == "repeats":
        v64 = synth.storage_to_f64(vals, "f16")
        X64 = synth.storage_to_f64(synth.to_storage(synth.normal((k, n), 96), "f16"), "f16")
        assert O.rel_fro(outs[0].cpu().numpy().astype(np.float64),
                         O.spmm_blockwise(m, k, b, rows, cols, v64, X64)) <= 5e-3


def test_multi_kernel_encoder_row_bitmap_and_fallbacks(monkeypatch):
    """The multi-kernel encoder's per-row ordering: rows placed through the column
    bitmap, rows with repeated (row, column) pairs and a row longer than 2048
    entries (both ranked pairwise) all give the oracle's plan, and Y matches the
    oracle (b = 1, 2048 x 4096 block grid)."""
    monkeypatch.setenv("SPMM_DYN_BUILDER", "multi")
    b, mb, kb, n = 1, 2048, 4096, 40
    g = np.random.default_rng(123)
    flat = g.choice(mb * kb, size=60000, replace=False)
    rows, cols = (flat // kb).astype(np.int32), (flat % kb).astype(np.int32)
    long_cols = g.choice(kb, size=3000, replace=False).astype(np.int32)  # row 7: 3000 entries
    rows = np.concatenate([rows[rows != 7], np.full(3000, 7, np.int32)])
    cols = np.concatenate([cols[flat // kb != 7], long_cols])
    rep = np.nonzero(np.isin(rows, [11, 500, 2047]))[0][:12]  # repeat some pairs of three rows
    rows, cols = np.concatenate([rows, rows[rep]]), np.concatenate([cols, cols[rep]])
    perm = g.permutation(len(rows))
    rows, cols = rows[perm], cols[perm]
    nnz = len(rows)
    vals = synth.to_storage(synth.normal((nnz, b, b), 124), "f16")
    Xs = synth.to_storage(synth.normal((kb * b, n), 125), "f16")
    h = spmm.DynamicHandle(mb * b, kb * b, b, nnz, "f16")
    ref = plan_ref.plan_from_coo(mb, kb, rows, cols, h.info()["group_rows"], h.info()["num_panels"])
    Y64 = O.spmm_blockwise(mb * b, kb * b, b, rows, cols, synth.storage_to_f64(vals, "f16"),
                           synth.storage_to_f64(Xs, "f16"))
    outs = []
    # the per-workgroup histogram count and scatter, then the global-atomic one
    for hist in (None, "0"):
        if hist:
            monkeypatch.setenv("SPMM_DYN_HIST", hist)
        else:
            monkeypatch.delenv("SPMM_DYN_HIST", raising=False)
        Y = torch.full((mb * b, n), float("nan"), dtype=torch.float16, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(torch.tensor([nnz], dtype=torch.int32, device="cuda"), dev(rows), dev(cols), dev(vals), dev(Xs), Y,
              status)
        torch.cuda.synchronize()
        assert status.item() == 0
        ex = h.export()
        for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
            assert np.array_equal(ex[key], ref[key]), key
        assert O.rel_fro(Y.cpu().numpy().astype(np.float64), Y64) <= 5e-3
        outs.append(Y)
    assert torch.equal(outs[0], outs[1])


def test_multi_kernel_encoder_status_words(monkeypatch):
    """The histogram encode reports capacity and index errors and leaves Y untouched."""
    monkeypatch.setenv("SPMM_DYN_BUILDER", "multi")
    b, m, k, n, cap = 4, 64, 80, 16, 3000
    h = spmm.DynamicHandle(m, k, b, cap, "f16")
    X = torch.ones((k, n), dtype=torch.float16, device="cuda")
    v = torch.ones((cap, b, b), dtype=torch.float16, device="cuda")
    g = np.random.default_rng(5)
    rows = g.integers(0, m // b, cap).astype(np.int32)
    cols = g.integers(0, k // b, cap).astype(np.int32)
    bad_row, bad_col = rows.copy(), cols.copy()
    bad_row[2999] = m // b
    bad_col[1234] = -1
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for r, c, nnz, want in [(rows, cols, cap + 1, spmm.ERR_CAPACITY), (bad_row, cols, cap, spmm.ERR_BAD_INDEX),
                            (rows, bad_col, cap, spmm.ERR_BAD_INDEX), (rows, cols, cap, 0)]:
        Y = torch.full((m, n), 3.0, dtype=torch.float16, device="cuda")
        h.run(torch.tensor([nnz], dtype=torch.int32, device="cuda"), dev(r), dev(c), v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == want
        if want:
            assert torch.all(Y == 3.0).item()
    ref = plan_ref.plan_from_coo(m // b, k // b, rows, cols, h.info()["group_rows"], h.info()["num_panels"])
    ex = h.export()
    for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
        assert np.array_equal(ex[key], ref[key]), key


# ---- the one-launch form: encode and multiply in one kernel (variant form 5)

def _call(h, nnz, r, c, v, X, Y, n, monkeypatch, fused):
    monkeypatch.setenv("SPMM_SPLIT_ALL", "1")  # the two-launch call runs the every-row split form
    monkeypatch.setenv("SPMM_DYN_FUSED", "1" if fused else "0")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, c, v, X, Y, status, n=n)
    torch.cuda.synchronize()
    return status.item()


@pytest.mark.parametrize("x,y,n", [("f16", "f16", 512), ("bf16", "f32", 70), ("f16", "f16", 1)])
def test_one_launch_call_equals_two_launch_call(x, y, n, monkeypatch):
    # ragged m, COO in random order with duplicates; both forms give the same
    # Y bit for bit and the same exported block-CSR, and match the oracle
    b, m, k = 16, 37 * 16 + 5, 48 * 16
    mb, kb = -(-m // b), k // b
    g = np.random.default_rng(7)
    nnz0 = 300
    rows = g.integers(0, mb, nnz0).astype(np.int32)
    cols = g.integers(0, kb, nnz0).astype(np.int32)
    vals = synth.to_storage(synth.normal((nnz0, b, b), 8), x)
    Xs = synth.to_storage(synth.normal((k, n), 9), x)
    max_nnz = 320
    r, c, v, nnz = _dyn_inputs(rows, cols, vals, max_nnz, b)
    ld = -(-n // 8) * 8  # leading dimensions of 16-byte multiples
    X = torch.zeros((k, ld), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[x]), device="cuda")
    X[:, :n] = dev(Xs)
    outs, exports = [], []
    for fused in (True, False):
        h = spmm.DynamicHandle(m, k, b, max_nnz, x, y=y)
        Y = torch.full((m, ld), float("nan"), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[y]), device="cuda")
        assert _call(h, nnz, r, c, v, X, Y, n, monkeypatch, fused) == 0
        outs.append(Y[:, :n])
        exports.append(h.export())
    assert torch.equal(outs[0], outs[1])
    for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
        assert np.array_equal(exports[0][key], exports[1][key]), key
    ref = O.spmm_expand(m, k, b, rows, cols, synth.storage_to_f64(vals, x), synth.storage_to_f64(Xs, x))
    got = outs[0].float().cpu().numpy().astype(np.float64)
    A = O.spmm_expand(m, k, b, rows, cols, np.abs(synth.storage_to_f64(vals, x)), np.abs(synth.storage_to_f64(Xs, x)))
    assert_elementwise(got, ref, A, 2 * k, y)


def test_one_launch_long_row_sorted_by_network(monkeypatch):
    # 3000 entries of one block row (duplicates of 64 columns) and a few
    # elsewhere: more than 8 keys per thread, so the row is sorted by the
    # bitonic network; equal to the two-launch call and the oracle
    b, m, k, n = 16, 8 * 16, 64 * 16, 96
    g = np.random.default_rng(11)
    rows = np.concatenate([np.full(3000, 5), g.integers(0, 8, 40)]).astype(np.int32)
    cols = g.integers(0, 64, len(rows)).astype(np.int32)
    vals = synth.to_storage(synth.integers((len(rows), b, b), 12, -1, 1), "f16")
    Xs = synth.to_storage(synth.integers((k, n), 13, -1, 1), "f16")
    max_nnz = 4096
    r, c, v, nnz = _dyn_inputs(rows, cols, vals, max_nnz, b)
    X = dev(Xs)
    outs = []
    for fused in (True, False):
        h = spmm.DynamicHandle(m, k, b, max_nnz, "f16", y="f32")
        Y = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
        assert _call(h, nnz, r, c, v, X, Y, n, monkeypatch, fused) == 0
        outs.append(Y)
    assert torch.equal(outs[0], outs[1])
    ref = O.spmm_expand(m, k, b, rows, cols, synth.storage_to_f64(vals, "f16"), synth.storage_to_f64(Xs, "f16"))
    assert np.array_equal(outs[0].cpu().numpy().astype(np.float64), ref)  # integer sums, exact in FP32


def test_one_launch_status_words_and_empty_call(monkeypatch):
    b, m, k, n = 16, 64, 64, 32
    h = spmm.DynamicHandle(m, k, b, 8, "f16")
    X = torch.ones((k, n), dtype=torch.float16, device="cuda")
    v = torch.ones((8, b, b), dtype=torch.float16, device="cuda")
    for rows, cols, nnz, want in [([0] * 8, [0] * 8, 9, spmm.ERR_CAPACITY), ([0] * 8, [0] * 8, -1, spmm.ERR_CAPACITY),
                                  ([0, 4] + [0] * 6, [0, 1] + [0] * 6, 2, spmm.ERR_BAD_INDEX),
                                  ([0, 1] + [0] * 6, [0, -1] + [0] * 6, 2, spmm.ERR_BAD_INDEX)]:
        Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
        r = torch.tensor(rows, dtype=torch.int32, device="cuda")
        c = torch.tensor(cols, dtype=torch.int32, device="cuda")
        nz = torch.tensor([nnz], dtype=torch.int32, device="cuda")
        assert _call(h, nz, r, c, v, X, Y, n, monkeypatch, True) == want
        assert torch.all(Y == 7.0).item()
    # an empty call writes zeros; then a valid one
    r = torch.zeros(8, dtype=torch.int32, device="cuda")
    Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
    assert _call(h, torch.tensor([0], dtype=torch.int32, device="cuda"), r, r, v, X, Y, n, monkeypatch, True) == 0
    assert torch.all(Y == 0).item()
    assert h.export()["row_ptr"].tolist() == [0] * (m // b + 1)
    Y = torch.full((m, n), 7.0, dtype=torch.float16, device="cuda")
    assert _call(h, torch.tensor([1], dtype=torch.int32, device="cuda"), r, r, v, X, Y, n, monkeypatch, True) == 0
    assert torch.all(Y[:16] == 16.0).item() and torch.all(Y[16:] == 0).item()


def test_one_launch_rule_at_the_dynamic_workload(monkeypatch):
    # m = k = 4096, n = 512, 8192 blocks at most: the rule runs the one-launch
    # form (no export of panels is made by it; the export derives them), and
    # its result equals the two-launch call's bit for bit
    monkeypatch.delenv("SPMM_DYN_FUSED", raising=False)
    b, m, k, n = 16, 4096, 4096, 512
    mb = kb = 256
    max_nnz = mb * kb // 8
    rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=5, dtype="f16")
    r, c, v, nnz = _dyn_inputs(rows, cols, vals, max_nnz, b)
    X = dev(synth.to_storage(synth.normal((k, n), 2), "f16"))
    outs = []
    for env in (None, "0"):
        if env is None:
            monkeypatch.delenv("SPMM_DYN_FUSED", raising=False)
        else:
            monkeypatch.setenv("SPMM_DYN_FUSED", env)
        h = spmm.DynamicHandle(m, k, b, max_nnz, "f16")
        Y = torch.full((m, n), float("nan"), dtype=torch.float16, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, X, Y, status)
        torch.cuda.synchronize()
        assert status.item() == 0
        outs.append((Y, h.export()))
    assert torch.equal(outs[0][0], outs[1][0])
    for key in ("row_ptr", "col_idx", "src", "panel_ptr"):
        assert np.array_equal(outs[0][1][key], outs[1][1][key]), key
