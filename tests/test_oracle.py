"""Pins of the FP64 oracle against facts fixed outside it (no GPU needed).

Each test checks the oracle against something other than itself: the paper's
elementwise definition evaluated by brute force, a library matmul in the dense
limit, exact integer arithmetic, permutation structure, linearity, column
separability and the paper's FLOP closed form (Section 3)."""
import os

import numpy as np
import pytest

from oracle import spmm_ref as O
from paper_2303_16999_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _random_case(g, m, k, n, b, d):
    mb, kb = -(-m // b), -(-k // b)
    M = (g.random((mb, kb)) < d).astype(np.uint8)
    W_full = g.standard_normal((mb * b, kb * b))  # values everywhere, also off-mask
    X = g.standard_normal((k, n))
    rr, cc = np.nonzero(M)
    vals = np.stack([W_full[r * b:(r + 1) * b, c * b:(c + 1) * b] for r, c in zip(rr, cc)]) if rr.size else np.zeros((0, b, b))
    return M, W_full[:m, :k], X, rr, cc, vals


@pytest.mark.parametrize("b", [1, 2, 3, 4, 8, 16, 32])
def test_expand_matches_bruteforce_definition(b):
    g = np.random.default_rng(100 + b)
    for trial in range(6):
        m, k, n = int(g.integers(1, 41)), int(g.integers(1, 41)), int(g.integers(1, 10))
        d = [0.0, 1.0, 0.3, 0.6, 0.1, 0.5][trial]
        M, W, X, rr, cc, vals = _random_case(g, m, k, n, b, d)
        Yb = O.spmm_bruteforce(M, W, X, b)
        Ye = O.spmm_expand(m, k, b, rr, cc, vals, X)
        Yw = O.spmm_blockwise(m, k, b, rr, cc, vals, X)
        np.testing.assert_allclose(Ye, Yb, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Yw, Yb, rtol=1e-12, atol=1e-12)


def test_density_one_is_dense_matmul():
    g = np.random.default_rng(7)
    m, k, n, b = 48, 40, 5, 8
    M = np.ones((6, 5), np.uint8)
    W = g.standard_normal((m, k))
    X = g.standard_normal((k, n))
    rr, cc = np.nonzero(M)
    vals = np.stack([W[r * b:(r + 1) * b, c * b:(c + 1) * b] for r, c in zip(rr, cc)])
    np.testing.assert_allclose(O.spmm_expand(m, k, b, rr, cc, vals, X), np.matmul(W, X), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(O.spmm_blockwise(m, k, b, rr, cc, vals, X), np.matmul(W, X), rtol=1e-12, atol=1e-12)


def test_density_zero_gives_zeros():
    X = np.random.default_rng(1).standard_normal((64, 3))
    Y = O.spmm_expand(32, 64, 16, [], [], np.zeros((0, 16, 16)), X)
    assert Y.shape == (32, 3) and not Y.any()
    assert O.rel_fro(np.zeros((32, 3)), Y) == 0.0
    assert O.rel_fro(np.full((32, 3), 0.5), Y) == 0.5


def test_block_permutation_of_identities_permutes_rows_exactly():
    b, nb, n = 4, 6, 7
    perm = np.random.default_rng(3).permutation(nb)
    rows = np.arange(nb)
    cols = perm
    vals = np.stack([np.eye(b)] * nb)
    X = np.random.default_rng(4).standard_normal((nb * b, n))
    Y = O.spmm_blockwise(nb * b, nb * b, b, rows, cols, vals, X)
    expect = np.concatenate([X[c * b:(c + 1) * b] for c in cols])
    assert np.array_equal(Y, expect)


def test_integer_data_is_exact():
    g = np.random.default_rng(11)
    m, k, n, b = 37, 29, 4, 8
    M, W, X, rr, cc, vals = _random_case(g, m, k, n, b, 0.5)
    W = np.round(W * 1.2)
    X = np.round(X * 1.2)
    vals = np.stack([np.round(v * 1.2) for v in vals])
    Y = O.spmm_expand(m, k, b, rr, cc, vals, X)
    # exact integer evaluation with Python ints, using the element mask directly
    Wi = W.astype(int).tolist()
    Xi = X.astype(int).tolist()
    for i in range(m):
        for j in range(n):
            s = sum(Wi[i][l] * Xi[l][j] for l in range(k) if M[i // b, l // b])
            assert Y[i, j] == s


def test_linearity_and_column_separability():
    g = np.random.default_rng(5)
    m, k, n, b = 40, 56, 6, 8
    M, W, X, rr, cc, v1 = _random_case(g, m, k, n, b, 0.4)
    v2 = g.standard_normal(v1.shape)
    X2 = g.standard_normal(X.shape)
    f = lambda v, x: O.spmm_blockwise(m, k, b, rr, cc, v, x)
    np.testing.assert_allclose(f(2.5 * v1 - 0.75 * v2, X), 2.5 * f(v1, X) - 0.75 * f(v2, X), atol=1e-12)
    np.testing.assert_allclose(f(v1, X + X2), f(v1, X) + f(v1, X2), atol=1e-12)
    S = np.array([5, 0, 3])
    np.testing.assert_allclose(O.spmm_blockwise_columns(m, k, b, rr, cc, v1, X, S), f(v1, X)[:, S], atol=0)


def test_duplicates_are_summed():
    b = 4
    X = np.random.default_rng(2).standard_normal((8, 3))
    v = np.random.default_rng(9).standard_normal((2, b, b))
    Y2 = O.spmm_expand(8, 8, b, [1, 1], [0, 0], v, X)
    Y1 = O.spmm_expand(8, 8, b, [1], [0], v[:1] + v[1:], X)
    np.testing.assert_allclose(Y2, Y1, atol=1e-12)


def test_partial_edge_blocks_ignore_out_of_range_part():
    b, m, k = 8, 13, 11
    vals = np.full((1, b, b), np.nan)
    vals[0, :5, :3] = 1.0  # only the in-range part of block (1, 1) is finite
    X = np.ones((k, 2))
    Y = O.spmm_expand(m, k, b, [1], [1], vals, X)
    assert np.all(Y[8:13] == 3.0) and np.all(Y[:8] == 0.0)


def test_flop_closed_form_golden():
    with open(os.path.join(GOLD, "flop_closed_form.txt")) as fh:
        lines = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    assert len(lines) >= 5
    for m, k, n, b, dn, dd, fl in (map(int, l) for l in lines):
        mb, kb = -(-m // b), -(-k // b)
        M = synth.block_mask(mb, kb, dn / dd, seed=0)
        assert O.useful_flops(m, k, n, b, M) == fl
        assert O.density(m, k, b, M) == dn / dd


def test_flop_count_with_partial_blocks_matches_element_mask():
    g = np.random.default_rng(8)
    m, k, b = 23, 18, 8
    M = (g.random((3, 3)) < 0.6).astype(np.uint8)
    elem = sum(int(M[i // b, l // b]) for i in range(m) for l in range(k))
    assert O.useful_flops(m, k, 3, b, M) == 2 * 3 * elem


def test_rel_fro_matches_definition():
    a = np.array([[3.0, 4.0]])
    assert O.rel_fro(a + np.array([[0.3, 0.4]]), a) == pytest.approx(0.1, rel=1e-15)


@pytest.mark.parametrize("b", [1, 3, 16, 64])
def test_ell_oracle_against_bruteforce_and_blockwise(b):
    from oracle import ell_ref as E
    from paper_2303_16999_amd import synth
    g = np.random.default_rng(300 + b)
    for trial in range(4):
        m, k, n = int(g.integers(1, 3 * b + 2)), int(g.integers(1, 3 * b + 2)), int(g.integers(1, 6))
        mb, kb = -(-m // b), -(-k // b)
        M = (g.random((mb, kb)) < [0.0, 1.0, 0.4, 0.7][trial]).astype(np.uint8)
        width = int(M.sum(1).max(initial=0)) + 1
        cols = synth.ell_from_mask(M, width, trial)
        vals = g.standard_normal((mb, width, b, b))
        X = g.standard_normal((k, n))
        Yb = E.ell_bruteforce(m, k, b, cols, vals, X)
        np.testing.assert_allclose(E.ell_spmm(m, k, b, cols, vals, X), Yb, rtol=1e-12, atol=1e-12)
        # the same blocks in CSR order through the Section 3 oracle
        rr, cc = np.nonzero(M)
        slot_of = {(r, int(cols[r, s])): s for r in range(mb) for s in range(width) if cols[r, s] >= 0}
        csr_vals = np.stack([vals[r, slot_of[(r, c)]] for r, c in zip(rr, cc)]) if rr.size else np.zeros((0, b, b))
        np.testing.assert_allclose(O.spmm_blockwise(m, k, b, rr, cc, csr_vals, X), Yb, rtol=1e-12, atol=1e-12)


def test_ell_empty_slots_contribute_nothing():
    from oracle import ell_ref as E
    cols = -np.ones((3, 4), np.int32)
    vals = np.full((3, 4, 2, 2), np.nan)  # never read
    assert not E.ell_spmm(6, 5, 2, cols, vals, np.ones((5, 3))).any()


def test_ell_from_mask_round_trip():
    from paper_2303_16999_amd import synth
    M = synth.block_mask(40, 30, 0.2, 7)
    cols = synth.ell_from_mask(M, int(M.sum(1).max()) + 3, 1)
    back = np.zeros_like(M)
    for r in range(M.shape[0]):
        for c in cols[r]:
            if c >= 0:
                back[r, c] = 1
    assert np.array_equal(back, M)
    assert ((cols >= 0).sum(1) == M.sum(1)).all()


def test_b64_expand_matches_bruteforce_definition():
    g = np.random.default_rng(164)
    for trial in range(3):
        m, k, n = int(g.integers(1, 150)), int(g.integers(1, 150)), int(g.integers(1, 4))
        M, W, X, rr, cc, vals = _random_case(g, m, k, n, 64, [1.0, 0.5, 0.3][trial])
        Yb = O.spmm_bruteforce(M, W, X, 64)
        np.testing.assert_allclose(O.spmm_expand(m, k, 64, rr, cc, vals, X), Yb, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(O.spmm_blockwise(m, k, 64, rr, cc, vals, X), Yb, rtol=1e-12, atol=1e-12)
