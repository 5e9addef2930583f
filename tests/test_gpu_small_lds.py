"""The LDS-staged kernels, b = 4 (panels of block rows share each chunk of
X in LDS; 4 x 4 x 4 matrix-core products) and b = 1 (panels of 64 rows, 512
columns per tile, dot products over pairs of nonzeros), against the FP64
oracle: ragged shapes across several chunks, panels and column tiles, every
16-bit dtype pair, integer data bit-exact, its row-per-wave variants bitwise equal to each other, empty rows,
dynamic calls equal to static plans bit for bit, and the kernel without LDS
within the rounding bound."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import TOL, Case, assert_elementwise, dev, round_like, y_f64

pytestmark = pytest.mark.gpu


def _run(c, monkeypatch, rw=None, lds=True):
    if rw is None:
        monkeypatch.delenv("SPMM_LDS_RW", raising=False)
    else:
        monkeypatch.setenv("SPMM_LDS_RW", str(rw))
    monkeypatch.setenv("SPMM_SMALL_LDS", "1" if lds else "0")
    plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y)
    vals, X, scales = c.device_inputs()
    plan.set_values(vals, scales)
    Y = c.new_Y()
    plan.run(X, Y, n=c.n)
    torch.cuda.synchronize()
    return Y


@pytest.mark.parametrize("w,y", [("f16", "f16"), ("bf16", "bf16"), ("f16", "f32"), ("bf16", "f32")])
@pytest.mark.parametrize("b,n", [(4, 1), (4, 37), (4, 100), (8, 37), (8, 100), (1, 1), (1, 37), (1, 100), (1, 600)])
def test_lds_ragged_shapes_match_oracle(w, y, b, n, monkeypatch):
    # k spans several chunks with a ragged tail; m leaves a partial panel
    c = Case(b * 301 + 3, 1500 + b // 2, n, b, 0.1, w=w, y=y, seed=400 + b + n)
    Y = _run(c, monkeypatch)
    got, ref = y_f64(Y, c), c.oracle()
    assert O.rel_fro(got, ref) <= TOL[y]
    assert_elementwise(got, ref, c.abs_oracle(), c.k, y)
    assert torch.isnan(Y[:, c.n:].float()).all().item()  # columns past n untouched


@pytest.mark.parametrize("b", [1, 4, 8])
def test_lds_integer_exact_and_row_variants_bitwise(b, monkeypatch):
    c = Case(b * 520, 2100, 130, b, 0.15, w="f16", seed=430 + b, integer=True)
    ref = round_like(c.oracle(), "f16")
    outs = []
    for rw in (8, 4, 2):
        Y = _run(c, monkeypatch, rw=rw)
        assert np.array_equal(y_f64(Y, c), ref), rw
        outs.append(Y)
    for Y in outs[1:]:
        assert torch.equal(Y[:, : c.n], outs[0][:, : c.n])


@pytest.mark.parametrize("b", [1, 4, 8])
def test_lds_empty_rows_density_zero_and_long_rows(b, monkeypatch):
    c = Case(b * 200, b * 700, 64, b, 0.3, w="bf16", seed=440 + b)
    mask = c.mask.copy()
    mask[5:40, :] = 0          # empty rows inside a panel
    mask[100, :] = 1           # a full row: many batches in every chunk
    c = Case(b * 200, b * 700, 64, b, 0.0, w="bf16", seed=440 + b, mask=mask)
    Y = _run(c, monkeypatch)
    assert O.rel_fro(y_f64(Y, c), c.oracle()) <= TOL["bf16"]
    assert torch.all(Y[5 * b: 40 * b, : c.n] == 0).item()
    z = Case(b * 64, b * 64, 40, b, 0.0, w="f16", seed=1)
    assert torch.all(_run(z, monkeypatch)[:, : z.n] == 0).item()


@pytest.mark.parametrize("b", [1, 4, 8])
def test_lds_against_kernel_without_lds(b, monkeypatch):
    c = Case(b * 260 + 1, b * 300 + 2, 260, b, 1 / 8, w="f16", y="f32", seed=450 + b)
    Yl = _run(c, monkeypatch, lds=True)
    Yv = _run(c, monkeypatch, lds=False)
    a, v = y_f64(Yl, c), y_f64(Yv, c)
    assert_elementwise(a, c.oracle(), c.abs_oracle(), c.k, "f32")
    assert O.rel_fro(a, v) <= 1e-6


@pytest.mark.parametrize("b", [1, 4, 8])
def test_lds_dynamic_equals_static(b, monkeypatch):
    monkeypatch.delenv("SPMM_LDS_RW", raising=False)
    c = Case(b * 180, b * 200, 96, b, 1 / 10, w="f16", seed=460 + b)
    Ys = _run(c, monkeypatch)
    max_nnz = len(c.rows) + 9
    perm = np.random.default_rng(3).permutation(len(c.rows))
    pad = max_nnz - len(c.rows)
    r = dev(np.concatenate([c.rows[perm], np.zeros(pad, np.int32)]).astype(np.int32))
    col = dev(np.concatenate([c.cols[perm], np.zeros(pad, np.int32)]).astype(np.int32))
    v = dev(np.concatenate([c.vals_store[perm], np.zeros((pad, b, b), c.vals_store.dtype)]))
    nnz = torch.tensor([len(c.rows)], dtype=torch.int32, device="cuda")
    h = spmm.DynamicHandle(c.m, c.k, b, max_nnz, "f16")
    _, X, _ = c.device_inputs()
    Yd = c.new_Y()
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    h.run(nnz, r, col, v, X, Yd, st, n=c.n)
    torch.cuda.synchronize()
    assert st.item() == 0
    assert torch.equal(Ys[:, : c.n], Yd[:, : c.n])


@pytest.mark.parametrize("b,n,dens", [(4, 1024, ((1 / 4, "1"), (1 / 16, "0"))),
                                      (4, 256, ((1 / 4, "0"),)),
                                      (8, 1024, ((1 / 4, "0"),)),
                                      (1, 1024, ((1 / 4, "1"), (1 / 8, "0"))),
                                      (1, 256, ((1 / 4, "0"),))])
def test_lds_chosen_by_density(b, n, dens, monkeypatch):
    """Without the override (and without tuning) the LDS kernels run from
    density 1/8 up at b = 4 and from 1/4 up at b = 1 once n reaches 1024 (b =
    1: 1/8 from n = 4096; both: 1/16 from n = 16384), never at smaller n;
    at b = 8 only from n = 16384.
    Both choices agree
    with the oracle (the dispatch is checked through results equal to the
    forced kernel's, bit for bit)."""
    monkeypatch.delenv("SPMM_LDS_RW", raising=False)
    monkeypatch.setenv("SPMM_AUTOTUNE", "0")  # the rule, not a measurement
    for d, lds in dens:
        c = Case(b * 300, b * 320 if b == 4 else 1280, n, b, d, w="f16", seed=470)
        monkeypatch.delenv("SPMM_SMALL_LDS", raising=False)
        plan = spmm.StaticPlan(c.m, c.k, c.b, c.mask, c.w, c.x, c.y)
        vals, X, _ = c.device_inputs()
        plan.set_values(vals)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        assert torch.equal(Y[:, : c.n], _run(c, monkeypatch, lds=lds == "1")[:, : c.n]), d
        assert O.rel_fro(y_f64(Y, c), c.oracle()) <= TOL["f16"]


@pytest.mark.parametrize("w", ["f16", "bf16"])
def test_b1_lds_dynamic_duplicates_past_one_batch(w, monkeypatch):
    """Dynamic calls may repeat an entry (summed), so a row can hold more than
    64 entries inside one chunk of 64 columns: the b = 1 LDS kernel then takes
    further batches within the chunk and reloads the row's batch at the next
    chunk. Integer data: exact against the FP64 oracle and equal to the kernel
    without LDS."""
    monkeypatch.delenv("SPMM_LDS_RW", raising=False)
    m, k, n, ldn = 150, 300, 600, 608  # 5 chunks (ragged tail), 2 column tiles (ragged)
    g = np.random.default_rng(7)
    base = np.argwhere(g.random((m, k)) < 1 / 8)
    rows = [base[:, 0]]
    cols = [base[:, 1]]
    rows += [np.full(150, 7), np.full(9, 7)]              # row 7: 150 entries in chunk 0, 9 in chunk 2
    cols += [g.integers(0, 64, 150), g.integers(128, 192, 9)]
    rows += [np.full(70, 70)]                             # row 70: 70 entries in chunk 1
    cols += [g.integers(64, 128, 70)]
    rows = np.concatenate(rows).astype(np.int32)
    cols = np.concatenate(cols).astype(np.int32)
    perm = g.permutation(len(rows))
    rows, cols = rows[perm], cols[perm]
    nnz_n = len(rows)
    vals = synth.to_storage(g.integers(-3, 4, (nnz_n, 1, 1)).astype(np.float64), w)
    X = synth.to_storage(g.integers(-3, 4, (k, n)).astype(np.float64), w)
    ref = O.spmm_expand(m, k, 1, rows, cols, synth.storage_to_f64(vals, w), synth.storage_to_f64(X, w))
    max_nnz = nnz_n + 5
    pad = max_nnz - nnz_n
    r = dev(np.concatenate([rows, np.zeros(pad, np.int32)]).astype(np.int32))
    c = dev(np.concatenate([cols, np.zeros(pad, np.int32)]).astype(np.int32))
    v = dev(np.concatenate([vals, np.zeros((pad, 1, 1), vals.dtype)]))
    nnz = torch.tensor([nnz_n], dtype=torch.int32, device="cuda")
    tdt = torch.float16 if w == "f16" else torch.bfloat16
    Xd = torch.zeros((k, ldn), dtype=tdt, device="cuda")
    Xd[:, :n] = dev(X)
    outs = []
    for lds in ("1", "0"):
        monkeypatch.setenv("SPMM_SMALL_LDS", lds)
        h = spmm.DynamicHandle(m, k, 1, max_nnz, w, y="f32")
        Y = torch.full((m, ldn), float("nan"), dtype=torch.float32, device="cuda")
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nnz, r, c, v, Xd, Y, st, n=n)
        torch.cuda.synchronize()
        assert st.item() == 0
        assert np.array_equal(Y[:, :n].cpu().numpy().astype(np.float64), ref), lds
        outs.append(Y)
    assert torch.equal(outs[0][:, :n], outs[1][:, :n])
