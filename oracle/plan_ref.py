"""Oracle for the static plan: block-CSR, row groups, cost-balanced panels and
the in-group column-major order.

TEST INFRASTRUCTURE ONLY: not imported by the library.

The paper's static partitioner splits the known nonzeros so that every part has
a balanced share (Section 3.2) but gives no rule. The rule below is this
library's reading, stated so that a CPU derivation and the GPU builder can agree
bit for bit (integer arithmetic only):

* block-CSR over the block mask M_hat (mb x kb): row_ptr[r+1] = row_ptr[r] +
  (ones in row r); col_idx lists each row's columns in ascending order.
* groups of R consecutive block rows: group g holds rows [g*R, min(g*R+R, mb)).
* group cost w_g = (blocks in g) + (rows in g); prefix C[0] = 0, C[g+1] = C[g] + w_g.
* P panels: panel_ptr[0] = 0, panel_ptr[P] = G, and for 0 < p < P
  panel_ptr[p] = the smallest g in [0, G] with C[g] >= floor(p * C[G] / P).
* order: inside each group the blocks are listed by (block column, block row)
  ascending; order[q] is the CSR position of the q-th listed block. Groups follow
  each other in ascending order.

For the dynamic mode the input is a COO list (row, col) that may be unsorted and
may repeat a position. Its canonical CSR order sorts entries by (row, col, input
index) and the in-group order by (col, row, input index); order[q] is then the
input index of the q-th listed entry.
"""
import numpy as np


def plan_from_mask(block_mask, R, P):
    """NumPy derivation of the plan (np.nonzero, cumsum, searchsorted, lexsort)."""
    M = np.asarray(block_mask) != 0
    mb, kb = M.shape
    rr, cc = np.nonzero(M)  # row-major enumeration == CSR order
    return _plan_from_sorted_coo(mb, rr.astype(np.int64), cc.astype(np.int64),
                                 np.arange(rr.size, dtype=np.int64), R, P)


def plan_from_coo(mb, kb, rows, cols, R, P):
    """Plan of a dynamic COO list; order[q] refers to input indices."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= mb or cols.min() < 0 or cols.max() >= kb):
        raise IndexError("COO index out of range")
    idx = np.arange(rows.size, dtype=np.int64)
    perm = np.lexsort((idx, cols, rows))  # primary key rows, then cols, then input index
    return _plan_from_sorted_coo(mb, rows[perm], cols[perm], idx[perm], R, P)


def _plan_from_sorted_coo(mb, rr, cc, src, R, P):
    if R < 1 or P < 1:
        raise ValueError("R and P must be positive")
    counts = np.bincount(rr, minlength=mb).astype(np.int64) if rr.size else np.zeros(mb, np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    G = -(-mb // R)
    g_lo = np.arange(G, dtype=np.int64) * R
    g_hi = np.minimum(g_lo + R, mb)
    w = (row_ptr[g_hi] - row_ptr[g_lo]) + (g_hi - g_lo)
    C = np.concatenate([[0], np.cumsum(w)]).astype(np.int64)
    targets = (np.arange(1, P, dtype=np.int64) * C[-1]) // P
    inner = np.searchsorted(C, targets, side="left")
    panel_ptr = np.concatenate([[0], inner, [G]]).astype(np.int64)
    grp = rr // R
    # sort by group, then column, then row, then source index (CSR position or input index)
    order_pos = np.lexsort((src, rr, cc, grp))
    order = src[order_pos]
    return {
        "row_ptr": row_ptr.astype(np.int32),
        "col_idx": cc.astype(np.int32),
        "src": src.astype(np.int32),
        "group_cost_prefix": C,
        "panel_ptr": panel_ptr.astype(np.int32),
        "order": order.astype(np.int32),
    }


def plan_loops(block_mask, R, P):
    """The same plan with plain Python loops (tiny inputs only)."""
    M = [[int(v != 0) for v in row] for row in np.asarray(block_mask).tolist()]
    mb = len(M)
    row_ptr = [0]
    col_idx = []
    for r in range(mb):
        for c, v in enumerate(M[r]):
            if v:
                col_idx.append(c)
        row_ptr.append(len(col_idx))
    G = (mb + R - 1) // R
    C = [0]
    for g in range(G):
        lo, hi = g * R, min(g * R + R, mb)
        C.append(C[-1] + (row_ptr[hi] - row_ptr[lo]) + (hi - lo))
    panel_ptr = [0]
    for p in range(1, P):
        t = (p * C[G]) // P
        g = 0
        while C[g] < t:
            g += 1
        panel_ptr.append(g)
    panel_ptr.append(G)
    order = []
    for g in range(G):
        lo, hi = g * R, min(g * R + R, mb)
        items = []
        for r in range(lo, hi):
            for pos in range(row_ptr[r], row_ptr[r + 1]):
                items.append((col_idx[pos], r, pos))
        items.sort()
        order.extend(pos for _, _, pos in items)
    return {"row_ptr": row_ptr, "col_idx": col_idx, "panel_ptr": panel_ptr, "order": order, "group_cost_prefix": C}
