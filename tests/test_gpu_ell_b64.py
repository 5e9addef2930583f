"""Blocked-ELL input and b = 64 blocks against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import ell_ref as E
from oracle import fp8_ref
from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import TOL, Case, dev, round_like, stored_f64, y_f64

pytestmark = pytest.mark.gpu


class EllCase:
    """A blocked-ELL problem: slot columns, slot values (stored), X (stored)."""

    def __init__(self, m, k, n, b, d, w="f16", x=None, y=None, seed=0, extra_width=2, integer=False):
        x = x or ("bf16" if w == "fp8" else w)
        y = y or x
        self.m, self.k, self.n, self.b, self.w, self.x, self.y = m, k, n, b, w, x, y
        mb, kb = -(-m // b), -(-k // b)
        self.mask = synth.block_mask(mb, kb, d, seed)
        self.width = int(self.mask.sum(1).max(initial=0)) + extra_width
        self.cols = synth.ell_from_mask(self.mask, self.width, seed + 1)
        shape = (mb * self.width, b, b)
        raw = synth.integers(shape, seed + 2) if integer else synth.normal(shape, seed + 2)
        self.scales = None
        if w == "fp8":
            self.vals_store, self.scales = synth.quantize_e4m3fn_blocks(raw)
            vals64 = fp8_ref.dequantize_blocks(self.vals_store, self.scales)
        else:
            self.vals_store = synth.to_storage(raw, w)
            vals64 = synth.storage_to_f64(self.vals_store, w)
        self.vals64 = vals64.reshape(mb, self.width, b, b)
        Xr = synth.integers((k, n), seed + 3) if integer else synth.normal((k, n), seed + 3)
        self.X_store = synth.to_storage(Xr, x)
        self.X64 = synth.storage_to_f64(self.X_store, x)

    def X_dev(self):
        ld = -(-self.n // 8) * 8
        X = torch.zeros((self.k, ld), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[self.x]), device="cuda")
        X[:, : self.n] = dev(self.X_store)
        return X

    def new_Y(self):
        ld = -(-self.n // 8) * 8
        return torch.full((self.m, ld), float("nan"), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[self.y]), device="cuda")

    def plan(self):
        p = spmm.StaticPlan.from_ell(self.m, self.k, self.b, self.cols, self.w, self.x, self.y)
        p.set_values_ell(dev(self.vals_store), dev(self.scales) if self.scales is not None else None)
        return p

    def run(self, plan):
        Y = self.new_Y()
        plan.run(self.X_dev(), Y, n=self.n)
        torch.cuda.synchronize()
        return stored_f64(Y[:, : self.n], self.y)

    def oracle(self):
        return E.ell_spmm(self.m, self.k, self.b, self.cols, self.vals64, self.X64)


@pytest.mark.parametrize("b", [1, 4, 16, 32, 64])
@pytest.mark.parametrize("w,x,y", [("f16", "f16", "f16"), ("bf16", "bf16", "f32"), ("fp8", "bf16", "bf16")])
def test_ell_plan_matches_oracle(b, w, x, y):
    c = EllCase(23 * b + (b // 3), 31 * b + (b // 2), 150, b, 1 / 5, w=w, x=x, y=y, seed=10 + b)
    err = O.rel_fro(c.run(c.plan()), c.oracle())
    assert err <= TOL[y], err


def test_ell_plan_fp32():
    c = EllCase(16 * 20 + 3, 16 * 17 + 5, 70, 16, 1 / 4, w="f32", seed=5)
    assert O.rel_fro(c.run(c.plan()), c.oracle()) <= 1e-5


@pytest.mark.parametrize("b", [16, 64])
def test_ell_plan_equals_mask_plan_bitwise(b):
    c = EllCase(40 * b, 30 * b, 257, b, 1 / 6, seed=21)
    ell_plan = c.plan()
    # the same blocks in CSR order through spmm_plan_static
    mb = c.cols.shape[0]
    rr, cc = np.nonzero(c.mask)
    slot_of = {(r, int(c.cols[r, s])): r * c.width + s for r in range(mb) for s in range(c.width) if c.cols[r, s] >= 0}
    order = np.array([slot_of[(r, col)] for r, col in zip(rr, cc)], np.int64)
    flat = c.vals_store.reshape(-1, b, b)
    mask_plan = spmm.StaticPlan(c.m, c.k, b, c.mask, "f16")
    mask_plan.set_values(dev(np.ascontiguousarray(flat[order])))
    assert np.array_equal(c.run(ell_plan), c.run(mask_plan))


def test_ell_integer_data_bit_exact_and_empty_rows():
    c = EllCase(16 * 33, 16 * 29, 96, 16, 1 / 8, seed=31, integer=True, extra_width=3)
    ref = c.oracle()
    assert np.abs(ref).max() <= 2048
    assert np.array_equal(c.run(c.plan()), round_like(ref, "f16"))


def test_ell_all_slots_empty():
    c = EllCase(100, 80, 40, 16, 0.0, seed=41, extra_width=2)
    assert (c.cols == -1).all()
    assert not c.run(c.plan()).any()


# ------------------------------------------------------------------ b = 64


@pytest.mark.parametrize("w,x,y", [("f16", "f16", "f16"), ("bf16", "bf16", "f32"), ("fp8", "f16", "f16"),
                                   ("fp8", "bf16", "f32")])
@pytest.mark.parametrize("variant", [0, 2, 4, 8])
def test_b64_matches_oracle(w, x, y, variant):
    c = Case(64 * 9 + 17, 64 * 11 + 40, 333, 64, 1 / 3, w=w, x=x, y=y, seed=50, scaled=(w == "fp8"))
    plan = spmm.StaticPlan(c.m, c.k, 64, c.mask, c.w, c.x, c.y, variant=variant)
    vals, X, scales = c.device_inputs()
    plan.set_values(vals, scales)
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    err = O.rel_fro(y_f64(Y, c), c.oracle())
    assert err <= TOL[y], err


def test_b64_variants_bitwise_and_integer_exact():
    c = Case(64 * 12 + 5, 64 * 10 + 3, 200, 64, 1 / 4, w="bf16", seed=60, integer=True)
    outs = []
    for v in (2, 4, 8):
        plan = spmm.StaticPlan(c.m, c.k, 64, c.mask, "bf16", variant=v)
        vals, X, _ = c.device_inputs()
        plan.set_values(vals)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        outs.append(y_f64(Y, c))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ref = c.oracle()
    assert np.abs(ref).max() <= 256
    assert np.array_equal(outs[0], round_like(ref, "bf16"))


def test_b64_autotune_and_transposed_plan():
    c = Case(64 * 8, 64 * 6 + 9, 512, 64, 1 / 3, w="f16", seed=70)
    plan = spmm.StaticPlan(c.m, c.k, 64, c.mask, "f16")
    vals, X, _ = c.device_inputs()
    plan.set_values(vals)
    Y = c.new_Y()
    best, times = plan.autotune(X, Y, n=c.n)
    # three tile widths of the plain row kernel (b = 64 has no pipelined form)
    assert best in times and sorted(times) == [2 + 256, 4 + 256, 8 + 256]
    # the transposed b = 64 plan against the oracle
    from oracle import train_ref as TR
    t = plan.transpose()
    dY64 = synth.storage_to_f64(synth.to_storage(synth.normal((c.m, c.n), 71), "f16"), "f16")
    dY = torch.zeros((c.m, c.n), dtype=torch.float16, device="cuda")
    dY[:] = dev(synth.to_storage(synth.normal((c.m, c.n), 71), "f16"))
    Z = torch.full((c.k, c.n), float("nan"), dtype=torch.float16, device="cuda")
    t.run(dY, Z)
    torch.cuda.synchronize()
    rt, ct, vt = TR.transpose_blocks(c.m, c.k, 64, c.rows, c.cols, c.vals64)
    assert O.rel_fro(stored_f64(Z, "f16"), O.spmm_blockwise(c.k, c.m, 64, rt, ct, vt, dY64)) <= 5e-3


def test_b64_full_size_sampled_columns():
    # m = k = 8192, n = 4096, b = 64, density 1/16, FP16: 128 sampled output columns
    c = Case(8192, 8192, 4096, 64, 1 / 16, w="f16", seed=80)
    plan = spmm.StaticPlan(c.m, c.k, 64, c.mask, "f16")
    vals, X, _ = c.device_inputs()
    plan.set_values(vals)
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    cols = np.random.default_rng(81).choice(c.n, 128, replace=False)
    got = stored_f64(Y[:, torch.from_numpy(cols).cuda()], "f16")
    assert O.rel_fro(got, c.oracle(cols)) <= 5e-3
