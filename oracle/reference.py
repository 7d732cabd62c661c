"""Acceptance oracle: oblique QR through a factorisation of A (test infrastructure only).

The oblique QR of a full-rank m x n Z (m >= n) in the inner product of an SPD A
is the unique pair Q (m x n, Q^T A Q = I) and R (n x n upper triangular with a
positive diagonal) with Z = QR (Section 1).  R is the Cholesky factor of
Z^T A Z (Section 2), and it is unique because that Cholesky factor is.

`chol_eqr` is the route of Algorithm 3 (Section 4): A = C^T C, Euclidean
Householder QR of W = C Z, then Q from C Q = Y.  Its orthogonality error is
bounded by c m n u ||A|| ||Q||^2 (Theorem 4.1), the best class in the paper,
and it never forms Z^T A Z, so it shares no step with the CholQR path under
test.  `eqr_syev` is Algorithm 4 (Section 5).  `stencil_eqr` is Algorithm 4
with the exact eigenbasis of the Dirichlet 7-point operator (the orthonormal
DST-I), used where A is only available matrix-free.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

from . import stencil as _st


def sign_fix(y: np.ndarray, r: np.ndarray):
    """Scale so that diag(R) > 0 (the unique factor of Section 1); Y columns follow."""
    s = np.sign(np.diag(r)).astype(np.float64)
    s[s == 0] = 1.0
    return y * s, s[:, None] * r


def householder_qr(w: np.ndarray):
    """Euclidean Householder QR (LAPACK geqrf/orgqr), reduced, positive diag(R)."""
    y, r = np.linalg.qr(w, mode="reduced")
    return sign_fix(y, r)


def chol_eqr(a: np.ndarray, z: np.ndarray):
    """CHOL-EQR (Algorithm 3, Section 4).

    C = chol(A) upper (A = C^T C); W = C Z; [Y, R] = qr(W); Q = C^{-1} Y.
    The listing's last step prints C \\ Z; the text of Section 4 and the
    triangular-solve error model solve C Q_j = Y_j, which is what is done."""
    a = np.asarray(a, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    c = np.linalg.cholesky(a).T              # upper, A = C^T C
    w = c @ z
    y, r = householder_qr(w)
    q = scipy.linalg.solve_triangular(c, y, lower=False, check_finite=False)
    return q, r


def eqr_syev(a: np.ndarray, z: np.ndarray):
    """EQR-SYEV (Algorithm 4, Section 5): A = V D V^T, W = D^{1/2} V^T Z, [Y,R] = qr(W), Q = V D^{-1/2} Y."""
    d, v = np.linalg.eigh(np.asarray(a, dtype=np.float64))
    x = v.T @ z
    w = np.sqrt(d)[:, None] * x
    y, r = householder_qr(w)
    u = y / np.sqrt(d)[:, None]
    return v @ u, r


def stencil_eqr(st, z: np.ndarray):
    """Algorithm 4 for the 7-point operator with its exact eigenbasis.

    The Dirichlet 7-point operator is diagonalised by the 3D orthonormal DST-I S
    (symmetric and its own inverse), with eigenvalues from `stencil.eigenvalues`.
    So V = S, W = D^{1/2} S Z, [Y, R] = qr(W), Q = S D^{-1/2} Y."""
    lam = _st.eigenvalues(st)                      # shape (nz, ny, nx)
    if np.any(lam <= 0):
        raise ValueError("stencil operator is not positive definite")
    m, n = z.shape
    shp = (st.nz, st.ny, st.nx)
    w = np.empty((m, n))
    for j in range(n):
        col = np.asarray(z[:, j], dtype=np.float64).reshape(shp)
        w[:, j] = (np.sqrt(lam) * scipy.fft.dstn(col, type=1, norm="ortho")).ravel()
    y, r = householder_qr(w)
    del w
    q = np.empty((m, n), order="F")
    for j in range(n):
        col = (y[:, j].reshape(shp) / np.sqrt(lam))
        q[:, j] = scipy.fft.dstn(col, type=1, norm="ortho").ravel()
    return q, r


def tridiag_eqr(t, z: np.ndarray):
    """CHOL-EQR (Algorithm 3) for a symmetric tridiagonal A with banded primitives: C = the upper
    bidiagonal Cholesky factor (A = C^T C, LAPACK pbtrf via scipy), W = C Z, [Y, R] = qr(W),
    Q = C^{-1} Y by banded back-substitution."""
    d = np.asarray(t.diag, dtype=np.float64)
    e = np.asarray(t.sub, dtype=np.float64)
    m = d.shape[0]
    ab = np.zeros((2, m))
    ab[0, 1:] = e                                  # upper form: superdiagonal, then diagonal
    ab[1, :] = d
    cb = scipy.linalg.cholesky_banded(ab, lower=False)
    z = np.asarray(z, dtype=np.float64)
    w = cb[1, :, None] * z
    w[:-1] += cb[0, 1:, None] * z[1:]              # W = C Z (C upper bidiagonal)
    y, r = householder_qr(w)
    q = scipy.linalg.solve_banded((0, 1), cb, y)
    return q, r


def oblique_qr(a_or_stencil, z: np.ndarray):
    """The oracle's answer (Q, R) for a dense SPD array, a Stencil7 or a Tridiag descriptor."""
    if hasattr(a_or_stencil, "nx"):
        return stencil_eqr(a_or_stencil, z)
    if hasattr(a_or_stencil, "sub"):
        return tridiag_eqr(a_or_stencil, z)
    return chol_eqr(a_or_stencil, z)


def gls(a_or_stencil, z: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Generalised least squares (Section 1): x minimising ||Z x - b||_A.

    Computed by whitening, independently of any oblique QR: with A = C^T C
    (Cholesky; for the stencil, C = D^{1/2} S from the exact DST-I eigenbasis),
    ||Z x - b||_A = ||C Z x - C b||_2, solved by LAPACK least squares.  b may hold
    several right-hand sides as columns."""
    z = np.asarray(z, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    if vec:
        b = b[:, None]
    if hasattr(a_or_stencil, "sub"):
        t = a_or_stencil
        m = t.m
        ab = np.zeros((2, m))
        ab[0, 1:] = t.sub
        ab[1, :] = t.diag
        cb = scipy.linalg.cholesky_banded(ab, lower=False)

        def cmul(x):
            out = cb[1, :, None] * x
            out[:-1] += cb[0, 1:, None] * x[1:]
            return out
        x = np.linalg.lstsq(cmul(z), cmul(b), rcond=None)[0]
        return x[:, 0] if vec else x
    if hasattr(a_or_stencil, "nx"):
        st = a_or_stencil
        lam = _st.eigenvalues(st)
        shp = (st.nz, st.ny, st.nx)

        def whiten(x):
            out = np.empty_like(x)
            for j in range(x.shape[1]):
                out[:, j] = (np.sqrt(lam) * scipy.fft.dstn(x[:, j].reshape(shp), type=1, norm="ortho")).ravel()
            return out
        cz, cb = whiten(z), whiten(b)
    else:
        c = np.linalg.cholesky(np.asarray(a_or_stencil, dtype=np.float64)).T
        cz, cb = c @ z, c @ b
    x = np.linalg.lstsq(cz, cb, rcond=None)[0]
    return x[:, 0] if vec else x
