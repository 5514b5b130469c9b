"""Helpers for the GPU parity tests (comparison logic only, no method arithmetic)."""
import numpy as np


def ulp(x):
    return np.spacing(np.abs(np.asarray(x, dtype=np.float64)))


def classify_mismatches(r_g, r_o, u_g, u_o, W_g, W_o):
    """Count index mismatches and check that each lies at a bin edge.

    A mismatch r_g != r_o at draw i is legitimate iff some edge e between the
    two indices (e in [min, max)) has |u_o[i] - W_o[e]| <= |u_g[i] - u_o[i]|
    + max|W_g - W_o| + 1 ulp(u_o[i]).  Returns (count, illegitimate indices).
    """
    r_g = np.asarray(r_g)
    r_o = np.asarray(r_o)
    mism = np.nonzero(r_g != r_o)[0]
    dW = float(np.max(np.abs(np.asarray(W_g) - np.asarray(W_o)))) if len(W_g) else 0.0
    bad = []
    for i in mism:
        lo, hi = sorted((int(r_g[i]), int(r_o[i])))
        tol = abs(u_g[i] - u_o[i]) + dW + ulp(u_o[i])
        edges = np.asarray(W_o[lo:hi])
        if edges.size == 0 or np.min(np.abs(u_o[i] - edges)) > tol:
            bad.append(int(i))
    return len(mism), bad


def assert_monotone_unit(W):
    W = np.asarray(W)
    assert np.all(np.diff(W) >= 0), "W not non-decreasing"
    assert W[-1] == 1.0, "W[M-1] != 1"
