"""Skewed patterns: long block rows split over a workgroup's waves (b = 16)."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import Case, round_like, y_f64

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
