"""Oracle for blocked-ELL input.

TEST INFRASTRUCTURE ONLY: not imported by the library.

Blocked ELL (the cuSPARSE layout the paper's GPU comparison sets aside,
Appendix B and Section 5) lists for every block row a fixed number of slots,
each a block-column index or -1 for an empty slot, with one b x b block of
values per slot. The product is the same SpMM as Section 3's, with the block
set given by the non-empty slots. Written in float64 straight from that
definition.
"""
import numpy as np


def ell_expand(m, k, b, ell_cols, ell_vals):
    """Dense m x k weight matrix: block (r, c) of every non-empty slot, clipped at m and k."""
    ell_cols = np.asarray(ell_cols)
    ell_vals = np.asarray(ell_vals, dtype=np.float64)
    mb = ell_cols.shape[0]
    kb = -(-k // b)
    W = np.zeros((mb * b, kb * b), dtype=np.float64)
    for r in range(mb):
        for s in range(ell_cols.shape[1]):
            c = int(ell_cols[r, s])
            if c < 0:
                continue
            W[r * b:(r + 1) * b, c * b:(c + 1) * b] += ell_vals[r, s]
    return W[:m, :k]


def ell_spmm(m, k, b, ell_cols, ell_vals, X):
    """Y = W X with W from the non-empty slots (float64)."""
    return ell_expand(m, k, b, ell_cols, ell_vals) @ np.asarray(X, dtype=np.float64)


def ell_bruteforce(m, k, b, ell_cols, ell_vals, X):
    """Element loop: Y[i, j] = sum over the slots of row i // b of the block's row i % b times X (tiny inputs)."""
    ell_cols = np.asarray(ell_cols)
    ell_vals = np.asarray(ell_vals, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[1]
    Y = np.zeros((m, n))
    for i in range(m):
        r, ii = divmod(i, b)
        for s in range(ell_cols.shape[1]):
            c = int(ell_cols[r, s])
            if c < 0:
                continue
            for t in range(b):
                l = c * b + t
                if l >= k:
                    continue
                for j in range(n):
                    Y[i, j] += ell_vals[r, s, ii, t] * X[l, j]
    return Y
