"""The matrix-free 7-point operator, as the oracle sees it (test infrastructure only).

Grid index p = x + nx (y + ny z); (A z)_p = center z_p + off * (sum of z_q over
the face neighbours q of p that lie in the grid).  With center = 6 + s and
off = -1 this is the Dirichlet 3D Laplacian (h = 1) plus s I.  The paper's own
sparse workload is a tridiagonal A (Section 8); the 3D stencil is the same kind
of O(mn) operator product.
"""
from __future__ import annotations

import numpy as np


def apply(st, x: np.ndarray) -> np.ndarray:
    """A @ x for x of shape (m,) or (m, k), by shifted slices of the grid."""
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    k = 1 if vec else x.shape[1]
    cols = x.reshape(st.m, k)
    out = np.empty((st.m, k), order="F")
    for j in range(k):
        c = cols[:, j].reshape(st.nz, st.ny, st.nx)
        y = st.center * c
        y[:, :, 1:] += st.off * c[:, :, :-1]
        y[:, :, :-1] += st.off * c[:, :, 1:]
        y[:, 1:, :] += st.off * c[:, :-1, :]
        y[:, :-1, :] += st.off * c[:, 1:, :]
        y[1:, :, :] += st.off * c[:-1, :, :]
        y[:-1, :, :] += st.off * c[1:, :, :]
        out[:, j] = y.ravel()
    return out[:, 0] if vec else out


def dense(st) -> np.ndarray:
    """Assemble A entry by entry from the neighbour rule (brute force, tiny grids)."""
    m = st.m
    a = np.zeros((m, m))
    for zz in range(st.nz):
        for yy in range(st.ny):
            for xx in range(st.nx):
                p = xx + st.nx * (yy + st.ny * zz)
                a[p, p] = st.center
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    qx, qy, qz = xx + dx, yy + dy, zz + dz
                    if 0 <= qx < st.nx and 0 <= qy < st.ny and 0 <= qz < st.nz:
                        a[p, qx + st.nx * (qy + st.ny * qz)] = st.off
    return a


def eigenvalues(st) -> np.ndarray:
    """Eigenvalues on the DST-I frequency grid, shape (nz, ny, nx).

    The 1D path operator with zero diagonal and unit off-diagonals on N points
    (Dirichlet) has eigenvalues 2 cos(pi k/(N+1)), k = 1..N, with the DST-I
    vectors; A = center I + off (T_x (+) T_y (+) T_z) is their Kronecker sum."""
    def one(nn):
        k = np.arange(1, nn + 1)
        return 2.0 * np.cos(np.pi * k / (nn + 1))
    ex, ey, ez = one(st.nx), one(st.ny), one(st.nz)
    return st.center + st.off * (ez[:, None, None] + ey[None, :, None] + ex[None, None, :])


def norm2(st) -> float:
    lam = eigenvalues(st)
    return float(lam.max())


def cond(st) -> float:
    lam = eigenvalues(st)
    return float(lam.max() / lam.min())
