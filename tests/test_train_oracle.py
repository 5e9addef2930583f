"""Pins of the training-direction oracle (transposed product, SDDMM) against
facts outside it: the dense transpose, the elementwise definition by brute
force, a library matmul, and the adjoint identity that ties SDDMM to the SpMM."""
import numpy as np
import pytest

from oracle import spmm_ref as O
from oracle import train_ref as T


def _case(g, m, k, n, b, d):
    mb, kb = -(-m // b), -(-k // b)
    M = (g.random((mb, kb)) < d).astype(np.uint8)
    rr, cc = np.nonzero(M)
    vals = g.standard_normal((rr.size, b, b))
    return M, rr, cc, vals, g.standard_normal((k, n)), g.standard_normal((m, n))


@pytest.mark.parametrize("b", [1, 3, 4, 16])
def test_transposed_blocks_expand_to_the_dense_transpose(b):
    g = np.random.default_rng(b)
    m, k = 5 * b + 2, 7 * b + 1
    M, rr, cc, vals, X, dY = _case(g, m, k, 3, b, 0.4)
    rt, ct, vt = T.transpose_blocks(m, k, b, rr, cc, vals)
    W = O.expand(m, k, b, rr, cc, vals)
    Wt = O.expand(k, m, b, rt, ct, vt)
    # edge parts of W outside m x k are dropped by expand; the transpose keeps exactly the in-range part
    np.testing.assert_array_equal(Wt, W.T)
    assert np.all(np.diff(rt * (m + 1) + ct) > 0)  # CSR order of W^T
    np.testing.assert_allclose(O.spmm_blockwise(k, m, b, rt, ct, vt, dY), W.T @ dY, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("b", [1, 2, 4, 8])
def test_sddmm_matches_bruteforce_and_dense_product(b):
    g = np.random.default_rng(10 + b)
    m, k, n = 3 * b + 1, 4 * b + 2, 5
    M, rr, cc, vals, X, dY = _case(g, m, k, n, b, 0.5)
    G = T.sddmm_blockwise(m, k, b, rr, cc, dY, X)
    dense = O.expand(m, k, b, rr, cc, G)
    np.testing.assert_allclose(dense, T.sddmm_bruteforce(M, dY, X, b), rtol=1e-12, atol=1e-12)
    elem = np.kron(M, np.ones((b, b)))[:m, :k]
    np.testing.assert_allclose(dense, (dY @ X.T) * elem, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("b", [1, 4, 16])
def test_sddmm_is_the_adjoint_of_the_spmm(b):
    # <G, V> summed over blocks equals <dY, (M o W) X> for any V on the same mask
    g = np.random.default_rng(20 + b)
    m, k, n = 6 * b, 5 * b, 7
    M, rr, cc, vals, X, dY = _case(g, m, k, n, b, 0.35)
    G = T.sddmm_blockwise(m, k, b, rr, cc, dY, X)
    lhs = float(np.sum(G * vals))
    rhs = float(np.sum(dY * O.spmm_blockwise(m, k, b, rr, cc, vals, X)))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs))
