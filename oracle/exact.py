"""Brute-force oblique QR at 50 significant digits (test infrastructure only).

For tiny inputs (m <= 32, n <= 6) the factors are computed from their
definition (Section 1 and Section 2): R is the Cholesky factor of the
normal-equation matrix Z^T A Z = R^T R, and Q = Z R^{-1}.  Every product of
two stored FP64 numbers is exact at this precision and each sum is rounded at
about 1e-50 relative, so the result, rounded back to FP64, is the exact
factorisation of the stored A and Z for all practical purposes.
"""
from __future__ import annotations

import mpmath
import numpy as np


def _mpmat(x):
    x = np.asarray(x, dtype=np.float64)
    return [[mpmath.mpf(float(v)) for v in row] for row in x]


def exact_gram(a, z, dps: int = 50):
    """Z^T A Z in mpmath (nested lists of mpf)."""
    with mpmath.workdps(dps):
        A, Z = _mpmat(a), _mpmat(z)
        m, n = len(Z), len(Z[0])
        B = [[mpmath.fsum(A[i][k] * Z[k][j] for k in range(m)) for j in range(n)] for i in range(m)]
        return [[mpmath.fsum(Z[k][i] * B[k][j] for k in range(m)) for j in range(n)] for i in range(n)]


def exact_oblique_qr(a, z, dps: int = 50):
    """(Q, R) as FP64 arrays, computed at `dps` digits from the definition."""
    z = np.asarray(z, dtype=np.float64)
    m, n = z.shape
    with mpmath.workdps(dps):
        G = exact_gram(a, z, dps)
        R = [[mpmath.mpf(0)] * n for _ in range(n)]
        for k in range(n):
            s = G[k][k] - mpmath.fsum(R[i][k] ** 2 for i in range(k))
            if s <= 0:
                raise ValueError("Z^T A Z is not positive definite at 50 digits")
            R[k][k] = mpmath.sqrt(s)
            for j in range(k + 1, n):
                R[k][j] = (G[k][j] - mpmath.fsum(R[i][k] * R[i][j] for i in range(k))) / R[k][k]
        Z = _mpmat(z)
        Q = [[mpmath.mpf(0)] * n for _ in range(m)]
        for row in range(m):
            for j in range(n):
                acc = Z[row][j] - mpmath.fsum(Q[row][i] * R[i][j] for i in range(j))
                Q[row][j] = acc / R[j][j]
        qf = np.array([[float(v) for v in r_] for r_ in Q])
        rf = np.array([[float(v) for v in r_] for r_ in R])
    return qf, rf
