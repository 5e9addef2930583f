"""The precision workload at its own shape: m = k = 16384, n = 2048, density
1/16, b = 16 and 32, weights N(0,1) times a per-block U(0.1, 10), BF16 X, in
BF16 and in FP8 E4M3 with per-block FP32 scales, BF16 and FP32 outputs
(FP32 accumulation throughout). 64 seeded columns are checked against the
FP64 oracle on the dequantized inputs: the relative Frobenius error within the
bound of the output type and every element within its rounding bound."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm
from gpu_cases import Case, TOL, assert_elementwise, y_f64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("w", ["bf16", "fp8"])
@pytest.mark.parametrize("b", [16, 32])
def test_precision_workload_sampled_columns(b, w):
    c = Case(16384, 16384, 2048, b, 1 / 16, w=w, x="bf16", y="bf16", seed=0, scaled=True)
    cols = np.sort(np.random.default_rng(44).choice(2048, 64, replace=False))
    ref, A = c.oracle(cols), c.abs_oracle(cols)
    vals, X, scales = c.device_inputs()
    # FP8 partials are scaled per block before they are added: one rounding more per block
    terms = 2 * c.k if w == "fp8" else c.k
    for y in ("bf16", "f32"):
        c.y = y
        plan = spmm.StaticPlan(c.m, c.k, b, c.mask, w, "bf16", y, n_hint=c.n)
        plan.set_values(vals, scales)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        got = y_f64(Y, c)[:, cols]
        err = O.rel_fro(got, ref)
        assert err <= TOL[y], (y, err)
        assert_elementwise(got, ref, A, terms, y)
        assert torch.isfinite(Y[:, : c.n]).all().item()
        plan.close()
