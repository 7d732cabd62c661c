"""Error measures and condition diagnostics (test infrastructure only).

Section 7 measures the loss of orthogonality as ||I - Q^T A Q||_2 and the
representativity (residual) error as ||Z - QR||_2 / ||Z||_2, or in the A-norm
||Z - QR||_A / ||Z||_A.  The Frobenius residual is reported as well.

A plain FP64 evaluation of Q^T A Q carries an error of order u ||A|| ||Q||^2
(the paper's conclusion notes that this is the best-case loss itself), so
`orth_loss_dd` evaluates it with error-free splitting of the operands
(products of slices accumulate exactly in FP64) and double-double sums, for
claims below about 1e-13.
"""
from __future__ import annotations

import numpy as np


def _apply(a, x):
    if hasattr(a, "nx"):
        from . import stencil
        return stencil.apply(a, x)
    if hasattr(a, "sub"):
        from . import tridiag
        return tridiag.apply(a, x)
    return a @ x


def orth_loss(a, q: np.ndarray) -> float:
    """||I - Q^T A Q||_2 in FP64."""
    g = q.T @ _apply(a, q)
    return float(np.linalg.norm(np.eye(q.shape[1]) - g, 2))


def residual_f(z, q, r) -> float:
    """||Z - QR||_F / ||Z||_F."""
    return float(np.linalg.norm(z - q @ r) / np.linalg.norm(z))


def residual_2(z, q, r) -> float:
    """||Z - QR||_2 / ||Z||_2."""
    return float(np.linalg.norm(z - q @ r, 2) / np.linalg.norm(z, 2))


def anorm(a, x) -> float:
    """||X||_A = ||A^{1/2} X||_2 = sqrt(lambda_max(X^T A X))."""
    g = x.T @ _apply(a, x)
    g = 0.5 * (g + g.T)
    return float(np.sqrt(max(np.linalg.eigvalsh(g).max(), 0.0)))


def residual_a(a, z, q, r) -> float:
    """||Z - QR||_A / ||Z||_A."""
    return anorm(a, z - q @ r) / anorm(a, z)


def r_forward_error(r, r_ref) -> float:
    return float(np.linalg.norm(r - r_ref) / np.linalg.norm(r_ref))


def diagnostics(a, z, q_ref, r_ref) -> dict:
    """kappa(A^{1/2} Z) = kappa(R) (Theorem 1.1), ||A|| ||Q||^2, kappa(Z), ||Q|| ||R||."""
    sr = np.linalg.svd(r_ref, compute_uv=False)
    sz = np.linalg.svd(z, compute_uv=False)
    qn = float(np.linalg.norm(q_ref, 2))
    if hasattr(a, "nx"):
        from . import stencil
        an = stencil.norm2(a)
    else:
        an = float(np.linalg.eigvalsh(a)[-1]) if a.shape[0] <= 4096 else float(np.linalg.norm(a, 2))
    return dict(kappa_ahalf_z=float(sr[0] / sr[-1]), a_q2=an * qn * qn, kappa_z=float(sz[0] / sz[-1]),
                q_r=qn * float(sr[0]), norm_a=an, norm_q=qn)


# ---- error-free evaluation of Q^T A Q --------------------------------------------------------

def _slices(x: np.ndarray, beta: int, axis: int, max_slices: int = 8):
    """x = sum of slices exactly; each slice has at most `beta` bits below its
    row (axis=1) or column (axis=0) maximum exponent."""
    out = []
    r = np.array(x, dtype=np.float64, copy=True)
    for _ in range(max_slices):
        mx = np.max(np.abs(r), axis=axis, keepdims=True)
        if not np.any(mx > 0):
            break
        e = np.ceil(np.log2(np.where(mx > 0, mx, 1.0))).astype(np.int64)
        sigma = np.ldexp(np.ones_like(mx), e + 53 - beta)
        sigma = np.where(mx > 0, sigma, 0.0)
        hi = (r + sigma) - sigma
        out.append(hi)
        r = r - hi
    return out


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _exact_matmul_dd(x, y):
    """x @ y as a double-double pair (hi, lo), from slice products that are exact in FP64."""
    k = x.shape[1]
    beta = (53 - int(np.ceil(np.log2(max(k, 2))))) // 2
    xs = _slices(x, beta, axis=1)
    ys = _slices(y, beta, axis=0)
    hi = np.zeros((x.shape[0], y.shape[1]))
    lo = np.zeros_like(hi)
    for xi in xs:
        for yj in ys:
            p = xi @ yj
            hi, e = _two_sum(hi, p)
            lo += e
    return hi, lo


def orth_loss_dd(a: np.ndarray, q: np.ndarray) -> float:
    """||I - Q^T A Q||_2 with Q^T A Q evaluated to about u^2 relative accuracy (dense A)."""
    ph, pl = _exact_matmul_dd(np.asarray(a, dtype=np.float64), q)
    gh, gl = _exact_matmul_dd(q.T, ph)
    gl = gl + q.T @ pl
    e = (gh - np.eye(q.shape[1])) + gl
    return float(np.linalg.norm(e, 2))
