"""Power-law model of the static sparse over dense speedup (PopSparse,
Section 5, "Will my application speed up?").

The paper summarises its static sweep by a power law in the feature size m,
the density d and the block size b, fitted to the measured ratio of static
sparse to dense FP16 TFLOP/s (both counting nonzero FLOPs, each best over the
batch size n): speedup ~ a * m^alpha * d^beta * b^gamma, with a predicted
speedup wherever that product exceeds 1. `fit` refits the same form by
least squares on log(speedup) to measurements of this library on MI355X
(bench.py --mode grid); `predict` evaluates a fit.

Host-side analysis only: nothing here runs on the GPU.
"""
import math

import numpy as np

# The paper's fit on its IPU sweep (Section 5): a, alpha (m), beta (d), gamma (b).
PAPER_FIT = {"a": 0.0013, "alpha": 0.59, "beta": -0.54, "gamma": 0.50}
# The same form fitted to this library on one MI355X (bench.py --mode grid, 96
# points; the C ABI's spmm_speedup_model carries these numbers).
MI355X_FIT = {"a": 0.07649, "alpha": -0.04109, "beta": -0.6541, "gamma": 0.7269}


def fit(points):
    """points: iterable of (m, d, b, speedup) with speedup > 0.
    Returns {"a", "alpha", "beta", "gamma", "r2", "rms_log_error", "points"}:
    the least-squares fit of log(speedup) = log(a) + alpha log(m) + beta log(d)
    + gamma log(b)."""
    pts = [(float(m), float(d), float(b), float(s)) for m, d, b, s in points if s and s > 0]
    if len(pts) < 4:
        raise ValueError("a power-law fit needs at least 4 points")
    A = np.array([[1.0, math.log(m), math.log(d), math.log(b)] for m, d, b, _ in pts])
    y = np.array([math.log(s) for _, _, _, s in pts])
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    res = y - A @ coef
    ss_tot = float(np.sum((y - y.mean()) ** 2))
    r2 = 1.0 - float(np.sum(res ** 2)) / ss_tot if ss_tot > 0 else 1.0
    return {"a": float(math.exp(coef[0])), "alpha": float(coef[1]), "beta": float(coef[2]),
            "gamma": float(coef[3]), "r2": r2, "rms_log_error": float(np.sqrt(np.mean(res ** 2))),
            "points": len(pts)}


def predict(m, d, b, model=None):
    """Predicted speedup a * m^alpha * d^beta * b^gamma (the paper's fit by default)."""
    f = PAPER_FIT if model is None else model
    return f["a"] * float(m) ** f["alpha"] * float(d) ** f["beta"] * float(b) ** f["gamma"]
