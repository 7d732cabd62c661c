"""The symmetric tridiagonal operator, as the oracle sees it (test infrastructure only).

A(i, i) = diag[i], A(i, i+1) = A(i+1, i) = sub[i]: the paper's sparse workload (a tridiagonal A,
Section 8).  Products by shifted slices; the dense matrix for small cross-checks.
"""
from __future__ import annotations

import numpy as np


def apply(t, x: np.ndarray) -> np.ndarray:
    """A @ x for x of shape (m,) or (m, k)."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(t.diag, dtype=np.float64)
    e = np.asarray(t.sub, dtype=np.float64)
    if x.ndim == 1:
        y = d * x
        y[1:] += e * x[:-1]
        y[:-1] += e * x[1:]
        return y
    y = d[:, None] * x
    y[1:] += e[:, None] * x[:-1]
    y[:-1] += e[:, None] * x[1:]
    return y


def dense(t) -> np.ndarray:
    d = np.asarray(t.diag, dtype=np.float64)
    e = np.asarray(t.sub, dtype=np.float64)
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
