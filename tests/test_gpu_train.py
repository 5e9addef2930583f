"""Training-direction products against the FP64 oracle: the transposed plan
(data gradient (M o W)^T dY) and the block-sampled product (weight gradient
(dY X^T) o M)."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from oracle import train_ref as TR
from paper_2303_16999_amd import spmm, synth
from gpu_cases import TOL, Case, dev, round_like, stored_f64

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _sampled_weight_gradient(monkeypatch):
    """The SDDMM tests below exercise the sampled kernels unless a test asks
    for the dense-GEMM form itself (a test's own setenv overrides this)."""
    monkeypatch.setenv("SPMM_SDDMM_DENSE", "0")


def _dY(c, seed, integer=False, code=None):
    """dY (m x n) in the plan's x dtype: device tensor (ld = n rounded to 8) and exact float64 values."""
    code = code or c.x
    v = synth.integers((c.m, c.n), seed) if integer else synth.normal((c.m, c.n), seed)
    st = synth.to_storage(v, code)
    ld = -(-c.n // 8) * 8
    t = torch.zeros((c.m, ld), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[code]), device="cuda")
    t[:, : c.n] = dev(st)
    return t, synth.storage_to_f64(st, code)


def _plan(c):
    plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y)
    vals, _, scales = c.device_inputs()
    plan.set_values(vals, scales)
    return plan


def _run_transposed(c, t, dY):
    Z = torch.full((c.k, -(-c.n // 8) * 8), float("nan"), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[c.y]), device="cuda")
    t.run(dY, Z, n=c.n)
    torch.cuda.synchronize()
    return stored_f64(Z[:, : c.n], c.y)


def _oracle_transposed(c, dY64):
    rt, ct, vt = TR.transpose_blocks(c.m, c.k, c.b, c.rows, c.cols, c.vals64)
    return O.spmm_blockwise(c.k, c.m, c.b, rt, ct, vt, dY64)


@pytest.mark.parametrize("b", [1, 4, 8, 16, 32])
@pytest.mark.parametrize("w,x,y", [("f16", "f16", "f16"), ("bf16", "bf16", "f32"), ("fp8", "bf16", "bf16"),
                                   ("f32", "f32", "f32")])
def test_transposed_plan_matches_oracle(b, w, x, y):
    # ragged: m, k not multiples of b, n not a multiple of any tile
    c = Case(37 * b + (b // 2 if b > 1 else 0), 53 * b + (b - 1), 203, b, 1 / 6, w=w, x=x, y=y, seed=7 + b,
             scaled=(w == "fp8"))
    plan = _plan(c)
    t = plan.transpose()
    assert t.info()["nnzb"] == plan.info()["nnzb"]
    dY, dY64 = _dY(c, 100 + b)
    err = O.rel_fro(_run_transposed(c, t, dY), _oracle_transposed(c, dY64))
    assert err <= TOL[y], err


@pytest.mark.parametrize("b", [4, 16, 32])
def test_transposed_plan_integer_data_bit_exact(b):
    c = Case(29 * b + 3, 41 * b + 1, 130, b, 1 / 5, w="f16", seed=21, integer=True)
    t = _plan(c).transpose()
    dY, dY64 = _dY(c, 22, integer=True)
    ref = _oracle_transposed(c, dY64)
    assert np.abs(ref).max() <= 2048
    assert np.array_equal(_run_transposed(c, t, dY), round_like(ref, "f16"))


def test_transposed_pattern_is_the_mask_transposed():
    c = Case(300, 500, 16, 16, 1 / 7, seed=3)
    t = _plan(c).transpose()
    ex = t.export()
    mb_t = -(-c.k // 16)
    rows = np.repeat(np.arange(mb_t), np.diff(ex["row_ptr"]))
    M_t = np.zeros((mb_t, -(-c.m // 16)), np.uint8)
    M_t[rows, ex["col_idx"]] = 1
    assert np.array_equal(M_t, c.mask.T)


def test_adjoint_identity():
    # <dY, (M o W) X> = <(M o W)^T dY, X> with FP32 data, at several tiles of every size
    c = Case(40 * 16 + 9, 70 * 16 + 5, 300, 16, 1 / 8, w="f32", seed=31)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    dY, dY64 = _dY(c, 32)
    Z = _run_transposed(c, plan.transpose(), dY)
    Y64 = stored_f64(Y[:, : c.n], "f32")
    lhs = float(np.sum(dY64 * Y64))
    rhs = float(np.sum(Z * c.X64))
    # |<a, y> - <a, y_exact>| <= ||a|| ||y - y_exact||, and each FP32 result is within 1e-5 relative of exact
    bound = 1e-5 * (np.linalg.norm(dY64) * np.linalg.norm(Y64) + np.linalg.norm(Z) * np.linalg.norm(c.X64))
    assert abs(lhs - rhs) <= bound, (lhs, rhs, bound)


def test_transposed_plan_owns_its_values():
    c = Case(200, 180, 64, 16, 1 / 4, seed=41)
    plan = _plan(c)
    t = plan.transpose()
    dY, dY64 = _dY(c, 42)
    want = _run_transposed(c, t, dY)
    plan.set_values(torch.zeros_like(c.device_inputs()[0]))  # later values on the source do not reach it
    plan.close()
    assert np.array_equal(_run_transposed(c, t, dY), want)


def test_transpose_of_empty_plan():
    c = Case(64, 96, 40, 16, 0.0, seed=1)
    plan = spmm.StaticPlan(c.m, c.k, 16, np.zeros_like(c.mask), "f16")
    plan.set_values(None)
    t = plan.transpose()
    dY, _ = _dY(c, 2)
    assert np.array_equal(_run_transposed(c, t, dY), np.zeros((c.k, c.n)))


# ------------------------------------------------------------------ SDDMM


def _sddmm(c, plan, dY, X, n=None):
    nnzb = plan.info()["nnzb"]
    G = torch.full((max(nnzb, 1), c.b, c.b), float("nan"), dtype=torch.float32, device="cuda")
    plan.sddmm(dY, X, G, n=c.n if n is None else n)
    torch.cuda.synchronize()
    return G[:nnzb].cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("b,tiled", [(1, "0"), (4, "0"), (8, "0"), (16, "0"), (16, "1"), (32, "0"), (32, "1")])
@pytest.mark.parametrize("dt", ["f16", "bf16"])
@pytest.mark.parametrize("n", [1, 31, 77, 300])
def test_sddmm_matches_oracle(b, tiled, dt, n, monkeypatch):
    # tiled: the form that stages a tile's dY and X rows in LDS (b = 16/32)
    monkeypatch.setenv("SPMM_SDDMM_TILED", tiled)
    c = Case(23 * b + 5, 31 * b + 11, n, b, 1 / 5, w=dt, seed=50 + b + n)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 60 + n)
    G = _sddmm(c, plan, dY, X)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    err = O.rel_fro(G, ref)
    assert err <= 1e-5, err
    # the parts of edge blocks outside m x k are exactly zero
    for e, (r, cc) in enumerate(zip(c.rows, c.cols)):
        rr, kk = c.m - r * b, c.k - cc * b
        if rr < b:
            assert not G[e, rr:, :].any()
        if kk < b:
            assert not G[e, :, kk:].any()


@pytest.mark.parametrize("b,tiled", [(1, "0"), (4, "0"), (8, "0"), (16, "0"), (16, "1"), (32, "0"), (32, "1")])
def test_sddmm_integer_data_bit_exact(b, tiled, monkeypatch):
    monkeypatch.setenv("SPMM_SDDMM_TILED", tiled)
    c = Case(17 * b + 7, 19 * b + 2, 250, b, 1 / 4, w="bf16", seed=70, integer=True)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 71, integer=True)
    G = _sddmm(c, plan, dY, X)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert np.array_equal(G, ref)


@pytest.mark.parametrize("tiled", ["0", "1"])
def test_sddmm_long_rows_and_dense_blocks(tiled, monkeypatch):
    monkeypatch.setenv("SPMM_SDDMM_TILED", tiled)
    # rows with more blocks than one task holds, a fully dense row, n spanning many 32-steps
    mb, kb, b = 12, 40, 16
    mask = synth.block_mask(mb, kb, 1 / 3, 80)
    mask[5, :] = 1
    c = Case(mb * b, kb * b, 517, b, 0.0, w="f16", seed=81, mask=mask)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 82)
    G = _sddmm(c, plan, dY, X)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert O.rel_fro(G, ref) <= 1e-5


@pytest.mark.parametrize("b", [1, 4, 8])
def test_sddmm_small_blocks_long_rows_ragged(b):
    # rows of several tasks (a task holds 64 / 16 / 8 blocks for b = 1 / 4 / 8),
    # a full row, partly filled MFMA groups, ragged m, k and n
    mb, kb = 9, 300 // b + 7
    mask = synth.block_mask(mb, kb, 0.35, 130 + b)
    mask[4, :] = 1
    mask[6, :] = 0
    c = Case(mb * b - (b > 1), kb * b - (b // 2), 203, b, 0.0, w="f16", seed=131 + b, mask=mask)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 132 + b)
    G = _sddmm(c, plan, dY, X)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert O.rel_fro(G, ref) <= 1e-5
    assert np.abs(G - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("b", [1, 4, 8])
def test_sddmm_small_blocks_many_tasks_sampled(b):
    # more than 32 tasks per compute unit (one task per wave over all of n), sampled blocks
    m = k = 4096
    c = Case(m, k, 64, b, {1: 1 / 8, 4: 1 / 4, 8: 1 / 3}[b], w="bf16", seed=140 + b)
    plan = _plan(c)
    nnzb = plan.info()["nnzb"]
    assert nnzb / {1: 64, 4: 16, 8: 8}[b] > 32 * 256
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 141 + b)
    G = torch.empty((nnzb, b, b), dtype=torch.float32, device="cuda")
    plan.sddmm(dY, X, G)
    torch.cuda.synchronize()
    pick = np.random.default_rng(142).choice(nnzb, 3000, replace=False)
    got = G[torch.from_numpy(pick).cuda()].cpu().numpy().astype(np.float64)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows[pick], c.cols[pick], dY64, c.X64)
    assert O.rel_fro(got, ref) <= 1e-5
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


def test_sddmm_n_zero_and_empty_plan():
    c = Case(100, 120, 40, 16, 1 / 3, w="f16", seed=90)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, _ = _dY(c, 91)
    G = _sddmm(c, plan, dY, X, n=0)
    assert not G.any()
    empty = spmm.StaticPlan(c.m, c.k, 16, np.zeros_like(c.mask), "f16")
    empty.set_values(None)
    G0 = torch.zeros((1, 16, 16), device="cuda")
    empty.sddmm(dY, X, G0, n=c.n)
    torch.cuda.synchronize()


def test_sddmm_with_fp8_weights():
    # the weight gradient needs only dY and X: an FP8-weight plan with BF16 data takes it too
    c = Case(30 * 16 + 3, 25 * 16 + 9, 150, 16, 1 / 4, w="fp8", x="bf16", seed=93, scaled=True)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 94)
    G = _sddmm(c, plan, dY, X)
    assert O.rel_fro(G, TR.sddmm_blockwise(c.m, c.k, 16, c.rows, c.cols, dY64, c.X64)) <= 1e-5


@pytest.mark.parametrize("b,w,x,y", [(64, "f16", "f16", "f16"), (16, "f32", "f32", "f32"), (16, "f16", "f16", "f32"),
                                     (4, "f32", "f32", "f32")])
def test_sddmm_rejects_unsupported_plans(b, w, x, y):
    c = Case(128, 128, 32, b, 1 / 2, w=w, x=x, y=y, seed=95)
    plan = _plan(c)
    G = torch.zeros((plan.info()["nnzb"], b, b), device="cuda")
    X = torch.zeros((c.k, 32), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[x]), device="cuda")
    dY = torch.zeros((c.m, 32), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[y]), device="cuda")
    with pytest.raises(spmm.SpmmError) as e:
        plan.sddmm(dY, X, G)
    assert e.value.status == spmm.ERR_UNSUPPORTED


def test_training_step_products_at_full_size_sampled():
    # m = k = 8192, n = 4096, b = 16, density 1/16, FP16: sampled blocks of dW, sampled columns of dX
    c = Case(8192, 8192, 4096, 16, 1 / 16, w="f16", seed=101)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 102)
    nnzb = plan.info()["nnzb"]
    G = torch.empty((nnzb, 16, 16), dtype=torch.float32, device="cuda")
    plan.sddmm(dY, X, G)
    t = plan.transpose()
    Z = torch.empty((c.k, c.n), dtype=torch.float16, device="cuda")
    t.run(dY, Z)
    torch.cuda.synchronize()
    rng = np.random.default_rng(103)
    pick = rng.choice(nnzb, 64, replace=False)
    ref = TR.sddmm_blockwise(c.m, c.k, 16, c.rows[pick], c.cols[pick], dY64, c.X64)
    assert O.rel_fro(G[torch.from_numpy(pick).cuda()].cpu().numpy(), ref) <= 1e-5
    cols = rng.choice(c.n, 24, replace=False)
    rt, ct, vt = TR.transpose_blocks(c.m, c.k, 16, c.rows, c.cols, c.vals64)
    refz = O.spmm_blockwise_columns(c.k, c.m, 16, rt, ct, vt, dY64, cols)
    assert O.rel_fro(stored_f64(Z[:, torch.from_numpy(cols).cuda()], "f16"), refz) <= 5e-3


def test_sddmm_many_tasks_one_wave_per_task():
    # more tasks than 32 per compute unit: each wave takes a whole task over n
    c = Case(8192, 8192, 96, 16, 1 / 4, w="bf16", seed=111)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 112)
    G1 = _sddmm(c, plan, dY, X)
    G2 = _sddmm(c, plan, dY, X)
    assert np.array_equal(G1, G2)
    ref = TR.sddmm_blockwise(c.m, c.k, 16, c.rows, c.cols, dY64, c.X64)
    assert O.rel_fro(G1, ref) <= 1e-5


def test_transpose_of_column_concentrated_pattern_has_split_rows():
    # all blocks in a few block columns: the transposed plan's rows are long and get split
    mb, kb, b = 300, 24, 16
    mask = synth.concentrated_mask(kb, mb, 1 / 8, 5).T.copy()  # concentrated in columns
    c = Case(mb * b, kb * b - 7, 180, b, 0.0, w="f16", seed=121, mask=mask)
    plan = _plan(c)
    t = plan.transpose()
    assert t.info()["num_split_rows"] > 0
    dY, dY64 = _dY(c, 122)
    err = O.rel_fro(_run_transposed(c, t, dY), _oracle_transposed(c, dY64))
    assert err <= 5e-3, err


def test_sddmm_on_concentrated_rows():
    # rows of hundreds of blocks: many tasks per row
    mb, kb, b = 20, 400, 16
    mask = synth.concentrated_mask(mb, kb, 1 / 5, 9)
    c = Case(mb * b, kb * b, 70, b, 0.0, w="bf16", seed=131, mask=mask)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 132)
    G = _sddmm(c, plan, dY, X)
    assert O.rel_fro(G, TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)) <= 1e-5


@pytest.mark.parametrize("b", [16, 32])
def test_tiled_sddmm_dense_tiles_ragged_edges_and_repeats(b, monkeypatch):
    """The tiled form: a tile full of blocks (more than one task per tile),
    tiles cut by m and k, n not a multiple of its 32-value chunks; the result
    against the oracle, repeatable bit for bit, and the rule's choice taken
    from density 1/4 at this size."""
    mb, kb = 512 // b * 2 + 3, 512 // b * 2 + 1
    mask = synth.block_mask(mb, kb, 1 / 3, 150 + b)
    mask[: 256 // b, : 256 // b] = 1  # one full tile
    c = Case(mb * b - 5, kb * b - 3, 333, b, 0.0, w="bf16", seed=151 + b, mask=mask)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 152 + b)
    monkeypatch.setenv("SPMM_SDDMM_TILED", "1")
    G1 = _sddmm(c, plan, dY, X)
    G2 = _sddmm(c, plan, dY, X)
    assert np.array_equal(G1, G2)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert O.rel_fro(G1, ref) <= 1e-5
    assert np.abs(G1 - ref).max() <= 1e-5 * np.abs(ref).max()
    monkeypatch.delenv("SPMM_SDDMM_TILED", raising=False)
    G3 = _sddmm(c, plan, dY, X)  # the rule: tiled at this density
    assert np.array_equal(G1, G3)


def test_tiled_sddmm_at_full_size_sampled(monkeypatch):
    # m = k = 8192, n = 4096, b = 16, density 1/4: sampled blocks against the oracle
    monkeypatch.setenv("SPMM_SDDMM_TILED", "1")
    c = Case(8192, 8192, 4096, 16, 1 / 4, w="f16", seed=160)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 161)
    nnzb = plan.info()["nnzb"]
    G = torch.empty((nnzb, 16, 16), dtype=torch.float32, device="cuda")
    plan.sddmm(dY, X, G)
    torch.cuda.synchronize()
    pick = np.random.default_rng(162).choice(nnzb, 256, replace=False)
    got = G[torch.from_numpy(pick).cuda()].cpu().numpy().astype(np.float64)
    ref = TR.sddmm_blockwise(c.m, c.k, 16, c.rows[pick], c.cols[pick], dY64, c.X64)
    assert O.rel_fro(got, ref) <= 1e-5



# ---- the weight gradient by a dense GEMM of dY X^T and a gather of the mask's blocks

@pytest.mark.parametrize("b", [1, 4, 8, 16, 32])
@pytest.mark.parametrize("dt", ["f16", "bf16"])
@pytest.mark.parametrize("n", [31, 300])
def test_sddmm_dense_gemm_matches_oracle(b, dt, n, monkeypatch):
    monkeypatch.setenv("SPMM_SDDMM_DENSE", "1")
    c = Case(23 * b + 5, 31 * b + 11, n, b, 1 / 5, w=dt, seed=150 + b + n)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 160 + n)
    G = _sddmm(c, plan, dY, X)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert O.rel_fro(G, ref) <= 1e-5
    for e, (r, cc) in enumerate(zip(c.rows, c.cols)):  # edge blocks: exactly zero outside m x k
        rr, kk = c.m - r * b, c.k - cc * b
        if rr < b:
            assert not G[e, rr:, :].any()
        if kk < b:
            assert not G[e, :, kk:].any()


def test_sddmm_dense_gemm_integer_data_bit_exact_over_several_panels(monkeypatch):
    # k = 65536: a 128 MiB FP32 panel holds 512 rows, so m = 1300 takes three
    # GEMMs and gathers; integer data is exact
    monkeypatch.setenv("SPMM_SDDMM_DENSE", "1")
    b = 16
    c = Case(1300, 65536, 24, b, 1 / 64, w="f16", seed=171, integer=True)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 172, integer=True)
    G = _sddmm(c, plan, dY, X)
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert np.array_equal(G, ref)


@pytest.mark.parametrize("b,d,dense", [(16, 1 / 4, True), (16, 1 / 16, False), (4, 1 / 16, True), (32, 1 / 8, False)])
def test_sddmm_rule_between_dense_gemm_and_sampled(b, d, dense, monkeypatch):
    # the rule by density and block size: the dense form's panel workspace
    # appears in the plan's memory only where it ran; both forms agree
    monkeypatch.delenv("SPMM_SDDMM_DENSE", raising=False)
    c = Case(64 * b, 48 * b, 200, b, d, w="f16", seed=180 + b)
    plan = _plan(c)
    _, X, _ = c.device_inputs()
    dY, dY64 = _dY(c, 181)
    before = plan.memory()[0]
    G = _sddmm(c, plan, dY, X)
    assert (plan.memory()[0] > before) == dense
    ref = TR.sddmm_blockwise(c.m, c.k, b, c.rows, c.cols, dY64, c.X64)
    assert O.rel_fro(G, ref) <= 1e-5
