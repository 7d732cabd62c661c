"""Emulated reduced-precision CholQR pass (test infrastructure only).

The paper analyses every step with one unit roundoff u (Section 1, notation).
The GPU library may run the operator product (dense A) or the Gram product
(stencil A) with operands split into bfloat16 slices and FP32 accumulation, and
keeps FP64 for the cross-tile sums, the Cholesky factorisation and the
triangular solve.  This module reproduces that arithmetic on the CPU so that
tests know the error level to expect: it predicts the level (within about
10x), not the bits, because accumulation order differs.

Slicing: s_0 = bf16(x), s_1 = bf16(x - s_0), ...  (round to nearest even,
through FP32).  A product of k-slice operands keeps the slice pairs with
i + j < k: 3 products for k = 2, 6 products for k = 3.  Products of two
bfloat16 values are exact in FP32; sums inside a K-tile of `kt` terms are
FP32, and tiles are summed in FP64.
"""
from __future__ import annotations

import numpy as np

from .variants import chol_info, trsm_right_upper

UNIT = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x2": 2.0 ** -24, "bf16x3": 2.0 ** -24}
NSLICE = {"bf16x2": 2, "bf16x3": 3}


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) through FP32; returned as float32 values."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split(x: np.ndarray, k: int):
    out = []
    r = np.asarray(x, dtype=np.float64)
    for _ in range(k):
        h = bf16(r)
        out.append(h)
        r = r - h.astype(np.float64)
    return out


def matmul(a: np.ndarray, b: np.ndarray, scheme: str, kt: int = 256) -> np.ndarray:
    """a @ b in the given scheme (fp64, fp32, bf16x2, bf16x3)."""
    if scheme == "fp64":
        return a @ b
    K = a.shape[1]
    if scheme == "fp32":
        a_s, b_s, pairs = [a.astype(np.float32)], [b.astype(np.float32)], [(0, 0)]
    else:
        k = NSLICE[scheme]
        a_s, b_s = split(a, k), split(b, k)
        pairs = [(i, j) for i in range(k) for j in range(k) if i + j < k]
    out = np.zeros((a.shape[0], b.shape[1]))
    for k0 in range(0, K, kt):
        k1 = min(K, k0 + kt)
        acc = np.zeros((a.shape[0], b.shape[1]), dtype=np.float32)
        for i, j in pairs:
            acc += a_s[i][:, k0:k1] @ b_s[j][k0:k1]
        out += acc.astype(np.float64)
    return out


def gram(a, z: np.ndarray, scheme: str, kt: int = 256, symmetric_blocks=None) -> np.ndarray:
    """G = Z^T (A Z): dense A -> reduced-precision A Z, FP64 Z^T W;
    stencil A -> exact FP64 stencil, reduced-precision Z^T W.

    symmetric_blocks = b (dense A only): the reading of steps 1-2 of Algorithm 1
    for a symmetric A that touches only A's upper block triangle.  With the
    rows cut into blocks of b, U holds the blocks strictly right of the
    diagonal and D the diagonal blocks (A = U + D + U^T):
        W_off = U Z (reduced precision),  W_sym = W_off + D Z (FP64),
        G = Z^T W_sym + W_off^T Z (FP64),
    which is Z^T A Z in exact arithmetic.  The rounding of the reduced-precision
    product then enters G as Z^T E + E^T Z, a symmetric perturbation."""
    if hasattr(a, "nx"):
        from . import stencil
        w = stencil.apply(a, z)
        return matmul(np.ascontiguousarray(z.T), w, scheme, kt)
    if symmetric_blocks:
        b = int(symmetric_blocks)
        m = a.shape[0]
        d = np.zeros_like(a)
        u = np.zeros_like(a)
        for t0 in range(0, m, b):
            t1 = min(m, t0 + b)
            d[t0:t1, t0:t1] = a[t0:t1, t0:t1]
            u[t0:t1, t1:] = a[t0:t1, t1:]
        w_off = matmul(u, z, scheme, kt)
        w_sym = w_off + d @ z
        return z.T @ w_sym + w_off.T @ z
    w = matmul(a, z, scheme, kt)
    return z.T @ w


def shift_for(g: np.ndarray, scheme: str, c: float) -> float:
    """s = c * u_p * max_i G_ii (max diag(G) <= ||G||_2 <= n max diag(G))."""
    return c * UNIT[scheme] * float(np.max(np.diag(g)))


def cholqr_pass(a, z: np.ndarray, scheme: str, shift_c: float = 1.0, max_retries: int = 3, kt: int = 256,
                symmetric_blocks=None):
    """One CHOLQR pass with a reduced-precision product, FP64 Cholesky with the
    shift-and-retry rule, FP64 substitution for Q.  A reduced-precision pass
    starts with s = shift_c u_p max diag(G); an FP64 pass starts unshifted and
    retries with shift_c u max diag(G); each further retry multiplies the
    constant by 10.  symmetric_blocks: see gram.

    Returns (Q, R, info, shift_used)."""
    g = gram(a, z, scheme, kt, symmetric_blocks)
    g = np.triu(g) + np.triu(g, 1).T          # the library reads the upper triangle
    c = shift_c if scheme != "fp64" else 0.0
    for attempt in range(max_retries + 1):
        s = shift_for(g, scheme, c) if c else 0.0
        r, info = chol_info(g + s * np.eye(g.shape[0]))
        if info == 0:
            return trsm_right_upper(z, r), r, 0, s
        c = (c * 10.0) if c else shift_c
    return None, r, info, s


def cholqr2(a, z: np.ndarray, scheme1: str, scheme2: str = "fp64", shift_c: float = 1.0, kt: int = 256,
            max_retries: int = 3, symmetric_blocks=None):
    q1, r1, info, s1 = cholqr_pass(a, z, scheme1, shift_c, max_retries, kt, symmetric_blocks)
    if info:
        return None, None, info
    q, r2, info, _ = cholqr_pass(a, q1, scheme2, shift_c, max_retries, kt, symmetric_blocks)
    if info:
        return None, None, info
    return q, np.triu(r2 @ r1), 0
