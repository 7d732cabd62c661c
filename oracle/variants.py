"""Per-algorithm FP64 CPU references (test infrastructure only).

Each function follows the algorithm's steps in the paper's order, in plain
NumPy, so that a GPU variant can be compared with the same algorithm's own FP64
behaviour (unstable variants are judged against themselves and against their
theorem's bound, not against the acceptance oracle).

* cholqr      Algorithm 1 (Section 2): B = A Z, C = Z^T B, R = chol(C), Q = Z R^{-1};
              for dense symmetric A, C may be formed from A's upper triangle (split_gram).
* cholqr2     Algorithm 1 applied twice, R = R2 R1 (the second pass plays the
              role of PRE-CHOLQR's R = U S, Algorithm 2, Section 3).
* pre_cholqr  Algorithm 2 (Section 3): [Y,S] = qr(Z), [Q,U] = CHOLQR(A,Y), R = U S.
* cgs, mgs_row, mgs_col, cgs2   Gram-Schmidt in the A inner product (Section 6;
              the row/column orientations of MGS are the two implementations
              described in the comments of Section 8).
* chol_info   right-looking Cholesky with a LAPACK-style failure index.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .reference import householder_qr


def chol_info(c: np.ndarray):
    """Upper Cholesky factor of symmetric C, textbook right-looking order.

    Returns (R, info): info = 0 on success, else the 1-based index k of the
    first pivot that is not positive (or is NaN); R is then only partial."""
    a = np.array(c, dtype=np.float64, copy=True)
    n = a.shape[0]
    r = np.zeros_like(a)
    for k in range(n):
        piv = a[k, k]
        if not (piv > 0.0):            # catches NaN too
            return r, k + 1
        rkk = np.sqrt(piv)
        r[k, k] = rkk
        r[k, k + 1:] = a[k, k + 1:] / rkk
        a[k + 1:, k + 1:] -= np.outer(r[k, k + 1:], r[k, k + 1:])
    return r, 0


def _apply(a, x):
    if hasattr(a, "nx"):
        from . import stencil
        return stencil.apply(a, x)
    if hasattr(a, "sub"):
        from . import tridiag
        return tridiag.apply(a, x)
    return a @ x


def trsm_right_upper(z: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Q = Z R^{-1}: each row q_i solves q_i R = z_i by substitution (Section 2)."""
    return scipy.linalg.solve_triangular(r, z.T, trans="T", lower=False, check_finite=False).T


def split_gram(a: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Z^T A Z for a dense symmetric A read in its upper triangle only: with T = triu(A, 1) + diag(A)/2,
    A = T + T^T exactly, so Z^T A Z = Z^T (T Z) + (T Z)^T Z, symmetric by construction."""
    t = np.triu(a, 1) + 0.5 * np.diag(np.diag(a))
    w = t @ z
    return z.T @ w + w.T @ z


def cholqr(a, z: np.ndarray, shift: float = 0.0, return_info: bool = False, gram: str = "sym"):
    """CHOLQR (Algorithm 1).  C = Z^T (A Z) is symmetric only in exact arithmetic:
    gram="sym" factors (C + C^T)/2; gram="upper" factors the symmetric matrix
    built from the upper triangle of C, which is what the listing's chol(C) reads
    (MATLAB's chol uses the upper triangle only); gram="split" (dense A) forms C from
    A's upper triangle as Z^T (T Z) + (T Z)^T Z (split_gram).  `shift` is added to
    the diagonal before the factorisation."""
    if gram == "split":
        c = split_gram(np.asarray(a), z)
    else:
        b = _apply(a, z)
        c = z.T @ b
    if gram == "sym":
        c = 0.5 * (c + c.T)
    elif gram == "upper":
        c = np.triu(c) + np.triu(c, 1).T
    elif gram != "split":
        raise ValueError(gram)
    if shift:
        c = c + shift * np.eye(c.shape[0])
    r, info = chol_info(c)
    if info:
        if return_info:
            return None, r, info
        raise np.linalg.LinAlgError(f"Cholesky pivot {info} not positive")
    q = trsm_right_upper(z, r)
    return (q, r, 0) if return_info else (q, r)


def cholqr2(a, z: np.ndarray, shift1: float = 0.0, gram: str = "sym"):
    """CHOLQR twice: (Q1, R1) = CHOLQR(A, Z); (Q, R2) = CHOLQR(A, Q1); R = R2 R1."""
    q1, r1 = cholqr(a, z, shift=shift1, gram=gram)
    q, r2 = cholqr(a, q1, gram=gram)
    return q, np.triu(r2 @ r1)


def pre_cholqr(a, z: np.ndarray, gram: str = "sym"):
    """PRE-CHOLQR (Algorithm 2)."""
    y, s = householder_qr(z)
    q, u = cholqr(a, y, gram=gram)
    return q, np.triu(u @ s)


def _anorm(a, v):
    return float(np.sqrt(v @ _apply(a, v)))


def cgs(a, z: np.ndarray):
    """Classical Gram-Schmidt: r_{1:j-1,j} = Q^T A z_j, v = z_j - Q r, r_jj = ||v||_A."""
    m, n = z.shape
    q = np.zeros((m, n))
    r = np.zeros((n, n))
    for j in range(n):
        v = np.array(z[:, j], dtype=np.float64)
        if j:
            r[:j, j] = q[:, :j].T @ _apply(a, z[:, j])
            v = v - q[:, :j] @ r[:j, j]
        r[j, j] = _anorm(a, v)
        q[:, j] = v / r[j, j]
    return q, r


def cgs2(a, z: np.ndarray):
    """Classical Gram-Schmidt with one reorthogonalisation (CGS2)."""
    m, n = z.shape
    q = np.zeros((m, n))
    r = np.zeros((n, n))
    for j in range(n):
        v = np.array(z[:, j], dtype=np.float64)
        if j:
            for _ in range(2):
                h = q[:, :j].T @ _apply(a, v)
                v = v - q[:, :j] @ h
                r[:j, j] += h
        r[j, j] = _anorm(a, v)
        q[:, j] = v / r[j, j]
    return q, r


def mgs_row(a, z: np.ndarray):
    """Row-oriented MGS: after q_i is final, p = A q_i once, then r_ij = p^T v_j, v_j -= r_ij q_i for j > i."""
    v = np.array(z, dtype=np.float64, order="F", copy=True)
    m, n = v.shape
    q = np.zeros((m, n))
    r = np.zeros((n, n))
    for i in range(n):
        r[i, i] = _anorm(a, v[:, i])
        q[:, i] = v[:, i] / r[i, i]
        if i + 1 < n:
            p = _apply(a, q[:, i])
            r[i, i + 1:] = p @ v[:, i + 1:]
            v[:, i + 1:] -= np.outer(q[:, i], r[i, i + 1:])
    return q, r


def mgs_col(a, z: np.ndarray):
    """Column-oriented MGS: for column j, r_ij = q_i^T A v (A inside the inner loop), v -= r_ij q_i."""
    m, n = z.shape
    q = np.zeros((m, n))
    r = np.zeros((n, n))
    for j in range(n):
        v = np.array(z[:, j], dtype=np.float64)
        for i in range(j):
            r[i, j] = q[:, i] @ _apply(a, v)
            v = v - r[i, j] * q[:, i]
        r[j, j] = _anorm(a, v)
        q[:, j] = v / r[j, j]
    return q, r


VARIANTS = {
    "cholqr": cholqr,
    "cholqr2": cholqr2,
    "pre_cholqr": pre_cholqr,
    "cgs": cgs,
    "cgs2": cgs2,
    "mgs_row": mgs_row,
    "mgs_col": mgs_col,
}
