"""Oracle for the two training-direction products of the block-sparse SpMM.

TEST INFRASTRUCTURE ONLY: not imported by the library.

The paper's product is Y = (M o W) X (Section 3), and it notes that PopSparse
implements further sparse operations besides it (opening of Section 3) with
sparse training as a motivation (Section 1). Differentiating the product
gives the other two operations a training step needs:

* data gradient   dX = (M o W)^T dY  -- the same block structure, transposed:
  block (r, c) of W becomes block (c, r) of W^T with its b x b values
  transposed;
* weight gradient dW = (dY X^T) o M  -- a sampled dense-dense product: only
  the b x b blocks of the mask are computed, G_rc = dY[rows of r] X[rows of c]^T.

Both are written here in float64 straight from these definitions.
"""
import numpy as np


def transpose_blocks(m, k, b, rows, cols, vals):
    """The nonzero blocks of W^T (shape k x m) in its block-CSR order, i.e.
    sorted by (block row of W^T, block column of W^T) = (c, r), each block's
    values transposed. Returns (rows_t, cols_t, vals_t)."""
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    cols = np.asarray(cols, dtype=np.int64).reshape(-1)
    vals = np.asarray(vals, dtype=np.float64).reshape(-1, b, b)
    order = np.lexsort((rows, cols))  # primary key: column of W
    return cols[order], rows[order], np.transpose(vals[order], (0, 2, 1)).copy()


def sddmm_blockwise(m, k, b, rows, cols, dY, X):
    """G_e = dY[rb : rb + b] @ X[cb : cb + b]^T for every listed block e = (r, c),
    as a [nnzb, b, b] array; the parts of edge blocks outside m x k are 0."""
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    cols = np.asarray(cols, dtype=np.int64).reshape(-1)
    dY = np.asarray(dY, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    G = np.zeros((rows.size, b, b), dtype=np.float64)
    for e, (r, c) in enumerate(zip(rows, cols)):
        r0, c0 = int(r) * b, int(c) * b
        r1, c1 = min(r0 + b, m), min(c0 + b, k)
        G[e, : r1 - r0, : c1 - c0] = dY[r0:r1] @ X[c0:c1].T
    return G


def sddmm_bruteforce(block_mask, dY, X, b):
    """Element loop over the mask: dW[i, j] = M_ij * sum_t dY[i, t] X[j, t] (tiny inputs)."""
    dY = np.asarray(dY, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    m, n = dY.shape
    k = X.shape[0]
    out = np.zeros((m, k), dtype=np.float64)
    for i in range(m):
        for j in range(k):
            if block_mask[i // b][j // b]:
                s = 0.0
                for t in range(n):
                    s += dY[i, t] * X[j, t]
                out[i, j] = s
    return out
