"""The allocation-free dynamic call (spmm_run_dynamic_noalloc) against the
handle-based spmm_run_dynamic on the same inputs: bit for bit, on two calls in
a row (the second smaller, so the shared device scratch holds the first call's
larger plan), and against the FP64 oracle; sizes beyond the scratch are
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import dev

pytestmark = pytest.mark.gpu


def _call(m, k, b, max_nnz, nnz, w, n, seed):
    mb, kb = m // b, k // b
    rows, cols, vals = synth.dynamic_call(mb, kb, b, max_nnz, seed=seed, dtype="f16", lo_frac=nnz / max_nnz)
    rows, cols, vals = rows[:nnz], cols[:nnz], vals[:nnz]
    pad = max_nnz - len(rows)
    r = dev(np.concatenate([rows, np.zeros(pad, np.int32)]).astype(np.int32))
    c = dev(np.concatenate([cols, np.zeros(pad, np.int32)]).astype(np.int32))
    v = dev(np.concatenate([vals, np.zeros((pad, b, b), vals.dtype)]))
    X_store = synth.to_storage(synth.normal((k, n), seed + 1), "f16")
    return rows, cols, vals, r, c, v, torch.tensor([len(rows)], dtype=torch.int32, device="cuda"), X_store


@pytest.mark.parametrize("b", [16, 4])
def test_noalloc_equals_handle_call_twice_second_smaller(b):
    m = k = 1024 if b == 16 else 512
    max_nnz = (m // b) * (k // b) // 8
    h = spmm.DynamicHandle(m, k, b, max_nnz, "f16")
    # first call: a full-capacity pattern and wide n; second: fewer blocks and narrower n
    for nnz, n, seed in ((max_nnz, 200, 31), (max_nnz // 3, 72, 47)):
        rows, cols, vals, r, c, v, nz, X_store = _call(m, k, b, max_nnz, nnz, "f16", n, seed)
        X = dev(X_store)
        Y_ref = torch.full((m, n), float("nan"), dtype=torch.float16, device="cuda")
        Y_na = torch.full((m, n), float("nan"), dtype=torch.float16, device="cuda")
        st_ref = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        st_na = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        h.run(nz, r, c, v, X, Y_ref, st_ref)
        spmm.run_dynamic_noalloc(m, k, b, max_nnz, nz, r, c, v, X, Y_na, st_na)
        torch.cuda.synchronize()
        assert st_ref.item() == 0 and st_na.item() == 0
        assert torch.equal(Y_ref, Y_na), (nnz, n)
        ref = O.spmm_blockwise(m, k, b, rows, cols, synth.storage_to_f64(vals, "f16"),
                               synth.storage_to_f64(X_store, "f16"))
        assert O.rel_fro(Y_na.cpu().numpy().astype(np.float64), ref) <= 5e-3
    h.close()


def test_noalloc_status_errors_leave_y_untouched():
    m = k = 256
    b, max_nnz = 16, 64
    rows, cols, vals, r, c, v, nz, X_store = _call(m, k, b, max_nnz, 40, "f16", 24, 5)
    X = dev(X_store)
    Y = torch.full((m, 24), 7.0, dtype=torch.float16, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    too_many = torch.tensor([max_nnz + 1], dtype=torch.int32, device="cuda")
    spmm.run_dynamic_noalloc(m, k, b, max_nnz, too_many, r, c, v, X, Y, st)
    torch.cuda.synchronize()
    assert st.item() == spmm.ERR_CAPACITY and torch.all(Y == 7.0).item()
    bad = r.clone()
    bad[3] = m // b  # a block row outside the grid
    spmm.run_dynamic_noalloc(m, k, b, max_nnz, nz, bad, c, v, X, Y, st)
    torch.cuda.synchronize()
    assert st.item() == spmm.ERR_BAD_INDEX and torch.all(Y == 7.0).item()


def test_noalloc_refuses_sizes_beyond_its_scratch():
    X = torch.zeros((4096, 8), dtype=torch.float16, device="cuda")
    Y = torch.zeros((4096, 8), dtype=torch.float16, device="cuda")
    i32 = torch.zeros(1 << 17, dtype=torch.int32, device="cuda")
    v = torch.zeros(16, dtype=torch.float16, device="cuda")
    with pytest.raises(spmm.SpmmError) as e:
        spmm.run_dynamic_noalloc(4096, 4096, 1, 1 << 17, i32[:1], i32, i32, v, X, Y, i32[:1])
    assert e.value.status == spmm.ERR_CAPACITY
    with pytest.raises(spmm.SpmmError) as e:  # b must divide k
        spmm.run_dynamic_noalloc(4096, 4090, 16, 64, i32[:1], i32, i32, v, X[:4090], Y, i32[:1])
    assert e.value.status == spmm.ERR_UNSUPPORTED
