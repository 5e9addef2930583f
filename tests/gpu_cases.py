"""Shared helpers for the GPU parity tests: seeded inputs on the device and
their FP64 oracle results."""
import numpy as np
import torch

from oracle import fp8_ref
from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth

TOL = {"f32": 1e-5, "f16": 5e-3, "bf16": 5e-3}


def dev(a, dtype_code=None):
    """numpy storage array -> CUDA tensor with the library's element type."""
    t = torch.from_numpy(np.ascontiguousarray(a))
    if a.dtype == np.uint16:
        t = t.view(torch.bfloat16)
    return t.cuda()


def stored_f64(t, code):
    """Exact float64 values of a device tensor of storage dtype `code`."""
    t = t.detach().cpu()
    if code == "bf16":
        return t.to(torch.float32).numpy().astype(np.float64)
    return t.to(torch.float64).numpy()


class Case:
    """A static SpMM problem: pattern, values (stored), X (stored), oracle inputs."""

    def __init__(self, m, k, n, b, d, w="f16", x=None, y=None, seed=0, integer=False, scaled=False,
                 mask=None, ldx=None, ldy=None):
        x = x or ("f16" if w == "fp8" else w)
        y = y or x
        self.m, self.k, self.n, self.b, self.w, self.x, self.y = m, k, n, b, w, x, y
        mb, kb = -(-m // b), -(-k // b)
        self.mask = synth.block_mask(mb, kb, d, seed) if mask is None else np.asarray(mask, np.uint8)
        self.rows, self.cols = synth.mask_coo(self.mask)
        nnz = len(self.rows)
        if integer:
            vals = synth.integers((nnz, b, b), seed + 1)
            X = synth.integers((k, n), seed + 2)
        else:
            vals = synth.scaled_block_values(nnz, b, seed + 1) if scaled else synth.normal((nnz, b, b), seed + 1)
            X = synth.normal((k, n), seed + 2)
        self.scales = None
        if w == "fp8":
            if integer:
                # small integers with unit scale encode exactly
                self.vals_store, self.scales = _encode_unit(vals), np.ones(nnz, np.float32)
            else:
                self.vals_store, self.scales = synth.quantize_e4m3fn_blocks(vals)
            self.vals64 = fp8_ref.dequantize_blocks(self.vals_store, self.scales)
        else:
            self.vals_store = synth.to_storage(vals, w)
            self.vals64 = synth.storage_to_f64(self.vals_store, w)
        self.vals_raw = vals.astype(np.float64)
        self.X_store = synth.to_storage(X, x)
        self.X64 = synth.storage_to_f64(self.X_store, x)
        self.ldx = ldx or -(-n // 8) * 8
        self.ldy = ldy or -(-n // 8) * 8

    def device_inputs(self):
        vals = dev(self.vals_store)
        Xfull = torch.zeros((self.k, self.ldx), dtype=spmm.torch_dtype(spmm.DTYPE_CODES[self.x]), device="cuda")
        Xfull[:, : self.n] = dev(self.X_store)
        scales = dev(self.scales) if self.scales is not None else None
        return vals, Xfull, scales

    def new_Y(self, fill=float("nan")):
        return torch.full((self.m, self.ldy), fill, dtype=spmm.torch_dtype(spmm.DTYPE_CODES[self.y]), device="cuda")

    def oracle(self, cols=None):
        if cols is None:
            return O.spmm_blockwise(self.m, self.k, self.b, self.rows, self.cols, self.vals64, self.X64)
        return O.spmm_blockwise_columns(self.m, self.k, self.b, self.rows, self.cols, self.vals64, self.X64, cols)

    def abs_oracle(self, cols=None):
        """(|M o W|) |X| in FP64 on the same columns: the scale of each output's
        rounding error."""
        X = np.abs(self.X64)
        V = np.abs(self.vals64)
        if cols is None:
            return O.spmm_blockwise(self.m, self.k, self.b, self.rows, self.cols, V, X)
        return O.spmm_blockwise_columns(self.m, self.k, self.b, self.rows, self.cols, V, X, cols)

    def run_static(self, group_rows=0, num_panels=0, n_hint=0, Y=None):
        plan = spmm.StaticPlan(self.m, self.k, self.b, self.mask, self.w, self.x, self.y, group_rows=group_rows,
                               num_panels=num_panels, n_hint=n_hint or self.n)
        vals, X, scales = self.device_inputs()
        plan.set_values(vals, scales)
        Y = self.new_Y() if Y is None else Y
        plan.run(X, Y, n=self.n)
        torch.cuda.synchronize()
        return plan, Y


def _encode_unit(vals):
    """E4M3FN codes of small integers (exact), scale 1."""
    grid = {0.0: 0x00, 1.0: 0x38, 2.0: 0x40, 3.0: 0x44, 4.0: 0x48}
    a = np.abs(vals)
    codes = np.vectorize(lambda v: grid[float(v)])(a).astype(np.uint8)
    return np.where(vals < 0, codes | 0x80, codes).astype(np.uint8)


def y_f64(Y, case):
    return stored_f64(Y[:, : case.n], case.y)


def round_like(Y64, code):
    """Round float64 results to the output dtype (nearest even), back to float64."""
    t = torch.from_numpy(Y64)
    dt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[code]
    return t.to(dt).to(torch.float64).numpy()


# unit roundoff and the smallest subnormal spacing of each output type
_UNIT = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}
_ETA = {"f32": 2.0 ** -150, "f16": 2.0 ** -25, "bf16": 2.0 ** -134}


def elementwise_bound(Y_ref, A, terms, code):
    """Per-element bound on |Y_dev - Y_ref| for a sum of `terms` products
    accumulated in FP32 in any order, then rounded once to `code`:
    |s - y| <= g A with g = t u32 / (1 - t u32) (A = (|W| |X|) of the element),
    and the final rounding adds u |s| + eta, with |s| <= |y| + g A."""
    u32 = 2.0 ** -24
    g = terms * u32 / (1.0 - terms * u32)
    u, eta = _UNIT[code], _ETA[code]
    return u * np.abs(Y_ref) + (1.0 + u) * g * A + eta


def assert_elementwise(Y_dev, Y_ref, A, terms, code):
    """Every element within elementwise_bound; reports the worst offender."""
    bound = elementwise_bound(Y_ref, A, terms, code)
    excess = np.abs(Y_dev - Y_ref) - bound
    if not np.all(excess <= 0):
        i = np.unravel_index(np.argmax(excess), excess.shape)
        raise AssertionError("element %s: got %r, oracle %r, bound %r (%d elements out of bound)"
                             % (i, Y_dev[i], Y_ref[i], bound[i], int(np.sum(excess > 0))))
