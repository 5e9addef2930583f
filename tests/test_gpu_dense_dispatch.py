"""Dense dispatch: a plan asks the speedup model at build time and, where the
model predicts the sparse kernels slower than a dense GEMM, keeps a dense copy
of M o W that the rule and the autotuner can run. Results against the FP64
oracle within the FP32-accumulation bound; the model's decision and the
candidate set are checked through the plan."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm
from gpu_cases import TOL, Case, assert_elementwise, y_f64

pytestmark = pytest.mark.gpu


def _plan(c, dense, variant=0):
    plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y, dense_dispatch=dense, variant=variant)
    vals, _, _ = c.device_inputs()
    plan.set_values(vals)
    return plan


def _run(c, plan):
    _, X, _ = c.device_inputs()
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    return Y


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "f32"), ("bf16", "bf16")])
def test_model_favours_dense_for_unstructured_sparsity(w, y, monkeypatch):
    # b = 1 at density 1/4: the model's ratio is far below 1
    c = Case(1000, 1100, 300, 1, 1 / 4, w=w, y=y, seed=500)
    plan = _plan(c, 1)
    ratio, dense = plan.dispatch()
    assert 0 < ratio < 1 and dense
    monkeypatch.setenv("SPMM_AUTOTUNE", "0")  # the rule follows the model: the dense GEMM runs
    Yr = _run(c, plan)
    Yd = _run(c, _plan(c, 1, variant=3 * 256))  # dense forced through the variant
    # the library GEMM may split its sums differently from run to run: compare
    # both against the oracle rather than bit for bit
    got, ref = y_f64(Yr, c), c.oracle()
    assert O.rel_fro(y_f64(Yd, c), ref) <= TOL[y]
    assert O.rel_fro(got, ref) <= TOL[y]
    assert_elementwise(got, ref, c.abs_oracle(), c.k, y)
    assert torch.isnan(Yr[:, c.n:].float()).all().item()  # columns past n untouched


def test_model_keeps_sparse_where_it_wins():
    c = Case(2048, 2048, 256, 16, 1 / 16, w="f16", seed=501)
    plan = _plan(c, 1)
    ratio, dense = plan.dispatch()
    assert ratio > 1 and not dense
    _, X, _ = c.device_inputs()
    _, times = plan.autotune(X, c.new_Y(), n=c.n)
    assert all((v >> 8) != 3 for v in times)  # no dense candidate
    # mode 2 keeps the copy anyway: the tuner measures it beside the sparse variants
    plan2 = _plan(c, 2)
    assert plan2.dispatch()[1]
    best, times2 = plan2.autotune(X, c.new_Y(), n=c.n)
    assert 3 * 256 in times2 and best in times2
    got = y_f64(_run(c, plan2), c)
    assert O.rel_fro(got, c.oracle()) <= TOL["f16"]


@pytest.mark.first_run_tuning
def test_first_run_tuning_chooses_between_dense_and_sparse():
    c = Case(2048, 2048, 512, 4, 1 / 8, w="f16", seed=502)
    plan = _plan(c, 2)
    Y = _run(c, plan)  # the first run measures every candidate, dense included
    v = plan.variant_for(c.n)
    assert v != 0
    got, ref = y_f64(Y, c), c.oracle()
    assert O.rel_fro(got, ref) <= TOL["f16"]
    assert_elementwise(got, ref, c.abs_oracle(), c.k, "f16")


def test_dense_copy_follows_new_values():
    c = Case(512, 640, 64, 4, 1 / 4, w="f16", seed=503)
    plan = _plan(c, 2, variant=3 * 256)
    Y1 = _run(c, plan)
    vals, _, _ = c.device_inputs()
    plan.set_values(-vals)  # replacing the values rebuilds the dense copy
    Y2 = _run(c, plan)
    ref = c.oracle()
    assert O.rel_fro(y_f64(Y1, c), ref) <= TOL["f16"]
    assert O.rel_fro(y_f64(Y2, c), -ref) <= TOL["f16"]


def test_dense_copy_of_empty_pattern_and_edge_blocks():
    # ragged m and k: the dense copy holds nothing past them
    c = Case(16 * 9 + 5, 16 * 7 + 3, 40, 16, 0.5, w="bf16", y="f32", seed=504)
    Y = _run(c, _plan(c, 2, variant=3 * 256))
    assert O.rel_fro(y_f64(Y, c), c.oracle()) <= TOL["f32"]
    z = Case(64, 64, 16, 16, 0.0, w="f16", seed=505)
    pz = spmm.StaticPlan(z.m, z.k, 16, np.zeros_like(z.mask), "f16", dense_dispatch=2, variant=3 * 256)
    pz.set_values(None)
    Yz = _run(z, pz)
    assert torch.all(Yz[:, : z.n] == 0).item()
