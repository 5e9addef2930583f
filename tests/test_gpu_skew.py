"""Skewed patterns: long block rows split over a workgroup's waves (b = 16)."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import Case, assert_elementwise, round_like, stored_f64, y_f64

pytestmark = pytest.mark.gpu


def _skewed_case(kind, m, k, n, d, w="f16", y=None, seed=0, integer=False):
    mb, kb = -(-m // 16), -(-k // 16)
    mask = synth.skewed_mask(mb, kb, d, 1.2, seed) if kind == "power" else synth.concentrated_mask(mb, kb, d, seed)
    x = "bf16" if w == "fp8" else None
    return Case(m, k, n, 16, 0.0, w=w, x=x, y=y, seed=seed, mask=mask, integer=integer,
                scaled=(w == "fp8" and not integer))


@pytest.mark.parametrize("kind", ["power", "concentrated"])
@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "f32"), ("fp8", "bf16")])
def test_split_rows_match_oracle(kind, w, y):
    c = _skewed_case(kind, 200 * 16 + 5, 150 * 16 + 3, 300, 1 / 10, w=w, y=y, seed=5)
    plan, Y = c.run_static()
    assert plan.info()["num_split_rows"] > 0
    err = O.rel_fro(y_f64(Y, c), c.oracle())
    assert err <= 5e-3, err


@pytest.mark.parametrize("kind", ["power", "concentrated"])
def test_split_rows_integer_data_bit_exact(kind):
    c = _skewed_case(kind, 96 * 16, 80 * 16, 160, 1 / 8, w="f16", seed=9, integer=True)
    plan, Y = c.run_static()
    assert plan.info()["num_split_rows"] > 0
    ref = c.oracle()
    assert np.abs(ref).max() <= 2048
    assert np.array_equal(y_f64(Y, c), round_like(ref, "f16"))


def test_split_and_unsplit_plans_agree_and_variants_are_bitwise(monkeypatch):
    c = _skewed_case("power", 160 * 16, 120 * 16, 333, 1 / 8, w="bf16", seed=11)
    outs = []
    for v in (2, 4, 8):
        plan = spmm.StaticPlan(c.m, c.k, 16, c.mask, "bf16", variant=v)
        vals, X, _ = c.device_inputs()
        plan.set_values(vals)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        assert plan.info()["num_split_rows"] > 0
        outs.append(Y)
    for Y in outs[1:]:
        assert torch.equal(outs[0][:, : c.n], Y[:, : c.n])
    monkeypatch.setenv("SPMM_SPLIT", "0")
    plan0, Y0 = c.run_static()
    assert plan0.info()["num_split_rows"] == 0
    assert O.rel_fro(y_f64(Y0, c), y_f64(outs[0], c)) <= 5e-3
    assert O.rel_fro(y_f64(outs[0], c), c.oracle()) <= 5e-3


@pytest.mark.parametrize("persist", ["0", "1"])
@pytest.mark.parametrize("count", [3, 40])
def test_grouped_launch_with_split_rows_equals_single_launches(count, persist, monkeypatch):
    monkeypatch.setenv("SPMM_GROUP_PERSIST", persist)
    # rows are split when longer than max(64, 4 x mean) blocks: k spans 200+ block columns
    cases = [_skewed_case("power" if i % 2 else "concentrated", (40 + 7 * (i % 3)) * 16, (200 + 10 * (i % 4)) * 16,
                          50 + 37 * (i % 5), 1 / 16, w="f16", seed=40 + i) for i in range(count)]
    plans, Xs, singles = [], [], []
    relu = [i % 2 for i in range(count)]
    for c in cases:
        plan, Ys = c.run_static()
        plans.append(plan)
        Xs.append(c.device_inputs()[1])
        singles.append(Ys[:, : c.n].clone())
    assert all(p.info()["num_split_rows"] > 0 for p in plans)
    g = spmm.Group(64)
    Ys = [c.new_Y() for c in cases]
    g.run(plans, Xs, Ys, ns=[c.n for c in cases], relu=relu)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        want = torch.clamp(singles[i], min=0) if relu[i] else singles[i]
        assert torch.equal(Ys[i][:, : c.n], want), i


def test_split_rows_deterministic():
    c = _skewed_case("concentrated", 64 * 16, 256 * 16, 4096, 1 / 8, w="f16", seed=3)
    plan, Y1 = c.run_static()
    _, X, _ = c.device_inputs()
    for _ in range(3):
        Y2 = c.new_Y()
        plan.run(X, Y2, n=c.n)
        torch.cuda.synchronize()
        assert torch.equal(Y1[:, : c.n], Y2[:, : c.n])


# ---- long rows cut into pieces over several workgroups (Appendix A.2's worst
# case: a partition whose nonzeros all sit in one row)

def _full_rows_mask(mb, kb, full_rows, d, seed):
    M = synth.block_mask(mb, kb, d, seed).copy()
    M[list(full_rows), :] = 1
    return M


def _plan_for(c, variant=0):
    plan = spmm.StaticPlan(c.m, c.k, 16, c.mask, c.w, c.x, c.y, variant=variant)
    vals, X, scales = c.device_inputs()
    plan.set_values(vals, scales)
    return plan, X


@pytest.mark.parametrize("n", [40, 300, 1000])
def test_rows_cut_into_pieces_integer_data_bit_exact(n, monkeypatch):
    # three full rows of 1000 blocks (4 pieces each), ragged m and k; FP32 Y
    # keeps the integer sums exact
    monkeypatch.setenv("SPMM_PIECES", "1")
    mask = _full_rows_mask(48, 1000, [0, 17, 47], 1 / 32, 21)
    c = Case(48 * 16 - 5, 1000 * 16 - 3, n, 16, 0.0, w="f16", y="f32", seed=21, mask=mask, integer=True)
    plan, X = _plan_for(c)
    before = plan.memory()[0]
    Y = c.new_Y()
    plan.run(X, Y, n=n)
    torch.cuda.synchronize()
    assert plan.info()["num_split_rows"] >= 3
    assert plan.memory()[0] > before  # the first run allocated the piece workspace
    assert np.array_equal(y_f64(Y, c), c.oracle())


def test_pieces_variants_bitwise_and_whole_rows_agree(monkeypatch):
    monkeypatch.setenv("SPMM_PIECES", "1")
    mask = _full_rows_mask(40, 600, [3, 4, 30], 1 / 16, 5)
    c = Case(40 * 16, 600 * 16, 333, 16, 0.0, w="bf16", y="f32", seed=5, mask=mask)
    outs = []
    for v in (2, 4, 8):
        plan, X = _plan_for(c, v)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        outs.append(Y)
    for Y in outs[1:]:
        assert torch.equal(outs[0][:, : c.n], Y[:, : c.n])
    monkeypatch.setenv("SPMM_PIECES", "0")  # long rows on one workgroup each
    plan0, X0 = _plan_for(c)
    before = plan0.memory()[0]
    Y0 = c.new_Y()
    plan0.run(X0, Y0, n=c.n)
    torch.cuda.synchronize()
    assert plan0.memory()[0] == before  # no pieces, no workspace
    ref, A = c.oracle(), c.abs_oracle()
    for Y in (outs[0], Y0):
        assert_elementwise(y_f64(Y, c), ref, A, 600 * 16, "f32")


def test_pieces_workspace_grows_and_runs_repeat(monkeypatch):
    # later runs, with fewer or more columns (the workspace grows), still
    # combine every piece
    monkeypatch.setenv("SPMM_PIECES", "1")
    mask = _full_rows_mask(32, 512, [0, 31], 1 / 16, 8)
    c = Case(32 * 16, 512 * 16, 1200, 16, 0.0, w="f16", y="f32", seed=8, mask=mask, integer=True)
    plan, X = _plan_for(c)
    ref = c.oracle()
    for n in (64, 1200, 64, 1200, 700):
        Y = c.new_Y()
        plan.run(X, Y, n=n)
        torch.cuda.synchronize()
        assert np.array_equal(stored_f64(Y[:, :n], "f32"), ref[:, :n]), n


@pytest.mark.parametrize("persist", ["0", "1"])
def test_grouped_pieces_with_a_repeated_plan_equal_single_runs(persist, monkeypatch):
    monkeypatch.setenv("SPMM_GROUP_PERSIST", persist)
    monkeypatch.setenv("SPMM_PIECES", "1")
    mask = _full_rows_mask(24, 700, [1, 2, 20], 1 / 16, 13)
    ns = (100, 257, 64, 513)
    cases = [Case(24 * 16, 700 * 16, n, 16, 0.0, w="f16", seed=13 + i, mask=mask) for i, n in enumerate(ns)]
    plan, _ = _plan_for(cases[0])  # one plan, four products with their own X
    other = _skewed_case("concentrated", 30 * 16, 400 * 16, 200, 1 / 4, w="f16", seed=7)
    plan2, X2 = _plan_for(other)
    Xs = [c.device_inputs()[1] for c in cases] + [X2]
    singles = []
    for c, X in zip(cases + [other], Xs):
        Y = c.new_Y()
        (plan2 if c is other else plan).run(X, Y, n=c.n)
        torch.cuda.synchronize()
        singles.append(Y[:, : c.n].clone())
    g = spmm.Group(8)
    Ys = [c.new_Y() for c in cases + [other]]
    g.run([plan] * 4 + [plan2], Xs, Ys, ns=[c.n for c in cases + [other]])
    torch.cuda.synchronize()
    for i, c in enumerate(cases + [other]):
        assert torch.equal(Ys[i][:, : c.n], singles[i]), i
    # the repeated plan's values are case 0's: check one product against the oracle
    c = cases[2]
    ref = O.spmm_blockwise(c.m, c.k, 16, cases[0].rows, cases[0].cols, cases[0].vals64, c.X64)
    assert O.rel_fro(y_f64(Ys[2], c), ref) <= 5e-3


@pytest.mark.parametrize("kind,n,cut", [("power", 1024, True), ("concentrated", 4096, False),
                                        ("concentrated", 1024, True)])
def test_pieces_rule_at_full_size(kind, n, cut, monkeypatch):
    # m = k = 8192, d = 1/16: the power law's split rows differ widely in
    # length (its long rows are cut); the concentrated pattern's are all full,
    # which the four-wave split balances where they give two workgroups per
    # CU (32 rows x 32 column tiles at n = 4096) and not where they give one
    # (n = 1024). Either way the result matches whole rows to rounding.
    c = _skewed_case(kind, 8192, 8192, n, 1 / 16, w="f16", seed=0)
    plan, X = _plan_for(c)
    before = plan.memory()[0]
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    assert (plan.memory()[0] > before) == cut  # the workspace exists only if pieces ran
    monkeypatch.setenv("SPMM_PIECES", "0")
    plan0, X0 = _plan_for(c)
    Y0 = c.new_Y()
    plan0.run(X0, Y0, n=c.n)
    torch.cuda.synchronize()
    assert O.rel_fro(y_f64(Y, c), y_f64(Y0, c)) <= 2e-3
    cols = np.arange(0, c.n, 37)
    ref = c.oracle(cols)
    assert_elementwise(y_f64(Y, c)[:, cols], ref, c.abs_oracle(cols), 8192, "f16")


def test_pieces_with_fp8_weights_and_block_scales(monkeypatch):
    # FP8 E4M3 weights with per-block FP32 scales, BF16 X: the pieces' partial
    # sums carry the scaled products; against the dequantized-input oracle
    monkeypatch.setenv("SPMM_PIECES", "1")
    mask = _full_rows_mask(40, 640, [2, 39], 1 / 16, 17)
    c = Case(40 * 16, 640 * 16, 200, 16, 0.0, w="fp8", x="bf16", y="f32", seed=17, mask=mask, scaled=True)
    plan, X = _plan_for(c)
    before = plan.memory()[0]
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    assert plan.memory()[0] > before
    assert_elementwise(y_f64(Y, c), c.oracle(), c.abs_oracle(), 640 * 16, "f32")


def test_grouped_pieces_apply_relu_in_the_fixup(monkeypatch):
    monkeypatch.setenv("SPMM_PIECES", "1")
    mask = _full_rows_mask(24, 600, [0, 11], 1 / 16, 19)
    cases = [Case(24 * 16, 600 * 16, n, 16, 0.0, w="f16", seed=19 + i, mask=mask) for i, n in enumerate((96, 130))]
    plan, _ = _plan_for(cases[0])
    Xs = [c.device_inputs()[1] for c in cases]
    singles = []
    for c, X in zip(cases, Xs):
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        singles.append(Y[:, : c.n].clone())
    g = spmm.Group(4)
    Ys = [c.new_Y() for c in cases]
    g.run([plan, plan], Xs, Ys, ns=[c.n for c in cases], relu=[1, 0])
    torch.cuda.synchronize()
    assert torch.equal(Ys[0][:, : cases[0].n], torch.clamp(singles[0], min=0))
    assert torch.equal(Ys[1][:, : cases[1].n], singles[1])
    assert (singles[0] < 0).any()  # the ReLU had something to clamp, cut rows included
    assert (Ys[0][:16, : cases[0].n] >= 0).all()  # block row 0 is a cut row
