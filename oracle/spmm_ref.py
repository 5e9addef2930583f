"""Oracle for the block-sparse SpMM of PopSparse (arXiv 2303.16999, Section 3).

TEST INFRASTRUCTURE ONLY: not imported by the library.

The paper defines the operation as Y = (M o W) * X with an element mask M derived
from a block mask M_hat of shape ceil(m/b) x ceil(k/b): M[i, j] = M_hat[i // b, j // b]
(Section 3, the SpMM equation). Y is m x n, X is k x n. Density d is the fraction
of ones in M and the useful work is 2*m*k*n*d FLOPs (Section 3, the paragraph
after the equation).

Sparse weights are given here the way the library receives them: a list of
nonzero blocks (block row r, block column c) with a b x b value array V_rc each.
Blocks at the right/bottom edge may extend past k/m; the part outside the matrix
is ignored (a reading: the paper only fixes the mask shape). A block listed
twice is summed (COO convention for the dynamic mode).

Every routine works in float64. Inputs stored as FP16/BF16/FP32/FP8 are upcast
exactly before they reach these routines.
"""
import numpy as np


def _as_blocks(rows, cols, vals, b):
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    cols = np.asarray(cols, dtype=np.int64).reshape(-1)
    vals = np.asarray(vals, dtype=np.float64).reshape(-1, b, b)
    if not (rows.shape[0] == cols.shape[0] == vals.shape[0]):
        raise ValueError("rows, cols and vals disagree on the number of blocks")
    return rows, cols, vals


def expand(m, k, b, rows, cols, vals):
    """Dense m x k float64 matrix (M o W) built from the nonzero blocks.

    This is the paper's (M o W) written out: every entry outside the listed
    blocks is zero; listed blocks are added in place (duplicates sum)."""
    rows, cols, vals = _as_blocks(rows, cols, vals, b)
    W = np.zeros((m, k), dtype=np.float64)
    for r, c, v in zip(rows, cols, vals):
        r0, c0 = int(r) * b, int(c) * b
        if r0 >= m or c0 >= k or r0 < 0 or c0 < 0:
            raise IndexError("block (%d, %d) lies outside the %d x %d matrix" % (r, c, m, k))
        r1, c1 = min(r0 + b, m), min(c0 + b, k)
        W[r0:r1, c0:c1] += v[: r1 - r0, : c1 - c0]
    return W


def spmm_expand(m, k, b, rows, cols, vals, X):
    """O1: Y = expand(W) @ X in float64 (Section 3 equation, dense form)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != k:
        raise ValueError("X must be k x n")
    return expand(m, k, b, rows, cols, vals) @ X


def spmm_bruteforce(block_mask, W_full, X, b):
    """O2: the elementwise definition, for tiny inputs only.

    block_mask is M_hat (ceil(m/b) x ceil(k/b)), W_full is the dense m x k value
    matrix W (its entries outside the mask may hold anything), X is k x n.
    Y[i, j] = sum_l M[i, l] * W[i, l] * X[l, j] with M[i, l] = M_hat[i // b, l // b].
    Masked-out entries contribute nothing even if X holds a non-finite value
    (sparse semantics: the product is never formed)."""
    block_mask = np.asarray(block_mask)
    W_full = np.asarray(W_full, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    m, k = W_full.shape
    n = X.shape[1]
    Y = np.zeros((m, n), dtype=np.float64)
    for i in range(m):
        for j in range(n):
            s = 0.0
            for l in range(k):
                if block_mask[i // b, l // b]:
                    s += W_full[i, l] * X[l, j]
            Y[i, j] = s
    return Y


def spmm_blockwise(m, k, b, rows, cols, vals, X):
    """O3: block-row by block-row, Y[r-rows] = sum over blocks of V_rc @ X[c-rows].

    Same sum as O1 but touching only nonzero blocks, so its cost is
    O(2 * n * nnz) as the paper's FLOP count assumes (Section 3)."""
    rows, cols, vals = _as_blocks(rows, cols, vals, b)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[1]
    Y = np.zeros((m, n), dtype=np.float64)
    for r, c, v in zip(rows, cols, vals):
        r0, c0 = int(r) * b, int(c) * b
        r1, c1 = min(r0 + b, m), min(c0 + b, k)
        Y[r0:r1] += v[: r1 - r0, : c1 - c0] @ X[c0:c1]
    return Y


def spmm_blockwise_columns(m, k, b, rows, cols, vals, X, col_idx):
    """O3 restricted to a subset of output columns.

    Exact by column separability: column j of Y depends only on column j of X,
    so Y[:, S] = f(W, X[:, S])."""
    X = np.asarray(X)[:, np.asarray(col_idx)]
    return spmm_blockwise(m, k, b, rows, cols, vals, X)


def rel_fro(Y_dev, Y_ref):
    """Relative Frobenius error ||Y_dev - Y_ref||_F / ||Y_ref||_F in float64.

    When Y_ref is all zero the error is max|Y_dev| (0 exactly when Y_dev is 0)."""
    Y_dev = np.asarray(Y_dev, dtype=np.float64)
    Y_ref = np.asarray(Y_ref, dtype=np.float64)
    den = np.linalg.norm(Y_ref)
    if den == 0.0:
        return float(np.max(np.abs(Y_dev))) if Y_dev.size else 0.0
    return float(np.linalg.norm(Y_dev - Y_ref) / den)


def useful_flops(m, k, n, b, block_mask):
    """2 * n * (number of ones of the element mask M).

    For full blocks this is the paper's 2*m*k*n*d (Section 3); with partial
    edge blocks only the in-range elements count."""
    block_mask = np.asarray(block_mask)
    mb, kb = block_mask.shape
    row_h = np.array([min(b, m - r * b) for r in range(mb)], dtype=np.int64)
    col_w = np.array([min(b, k - c * b) for c in range(kb)], dtype=np.int64)
    elems = int((block_mask.astype(np.int64) * row_h[:, None] * col_w[None, :]).sum())
    return 2 * n * elems


def density(m, k, b, block_mask):
    """d = sum_ij M_ij / (m * k) (Section 3)."""
    return useful_flops(m, k, 1, b, block_mask) / (2.0 * m * k)
