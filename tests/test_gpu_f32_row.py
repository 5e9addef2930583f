"""The row-wise FP32 kernel (b = 16/32, FP32 W, X and Y) against the FP64
oracle."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm
from gpu_cases import Case, round_like, y_f64

pytestmark = pytest.mark.gpu


def _run(c):
    plan, Y = c.run_static()
    return y_f64(Y, c)


@pytest.mark.parametrize("b", [16, 32])
@pytest.mark.parametrize("n", [1, 33, 100, 515])
def test_row_f32_matches_oracle(b, n):
    c = Case(b * 23 + 7, b * 19 + 5, n, b, 1 / 4, w="f32", seed=200 + n + b)
    err = O.rel_fro(_run(c), c.oracle())
    assert err <= 1e-5, err


@pytest.mark.parametrize("b", [16, 32])
def test_row_f32_integer_exact(b):
    c = Case(b * 30 + 3, b * 26 + 9, 130, b, 1 / 5, w="f32", seed=220 + b, integer=True)
    row = _run(c)
    assert np.array_equal(row, round_like(c.oracle(), "f32"))
    assert np.array_equal(_run(c), row)


def test_row_f32_small_config_and_empty_rows():
    # m = k = 1024, n = 64, b = 16, d = 1/16 (the small FP32 case); rows without blocks are 0
    c = Case(1024, 1024, 64, 16, 1 / 16, w="f32", seed=0)
    c.mask[3, :] = 0
    c.__init__(1024, 1024, 64, 16, 0.0, w="f32", seed=0, mask=c.mask)
    Y = _run(c)
    assert O.rel_fro(Y, c.oracle()) <= 1e-5
    assert not Y[48:64].any()
