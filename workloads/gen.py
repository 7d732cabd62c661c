"""Seeded test-matrix generators.

The constructions follow Section 7 (stability experiments) of Lowery & Langou:

* A = V diag(d) V^T with V a random orthogonal matrix and log10 d_ii evenly
  spaced from 0 to log10 kappa(A), so d runs from 1 to kappa(A);
* Z = U diag(s) W^T with log10 s_ii evenly spaced from 0 to log10 kappa(Z),
  U either random orthonormal (Case 4) or chosen eigenvectors of A
  (Cases 1, 2, 3 and 5) and W a random orthogonal n x n matrix.

The paper draws V as orth(randn(m)).  `haar` reproduces that distribution by a
QR factorisation of a Gaussian matrix with the sign of diag(R) fixed.  For
m beyond a few thousand that costs O(m^3) host flops, so `butterfly` builds a
dense random orthogonal V from rounds of random permutations and
block-diagonal Haar blocks instead (O(m^2 b) flops for block size b).

Every draw comes from numpy.random.default_rng(SeedSequence([15171, cfg, i])).
Nothing here computes a factorisation of Z in the A inner product.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterable, Optional

import numpy as np

BASE_SEED = 15171

__all__ = [
    "BASE_SEED", "rng_for", "logspace_to", "haar", "Butterfly", "butterfly",
    "spd_from_eigs", "spd_from_eigs_torch", "dense_spd", "dense_spd_device", "tall_skinny", "gaussian_scaled",
    "paper_case", "Stencil7", "laplacian7", "Tridiag", "laplacian1d", "BatchInstance", "batch_plan",
    "batch_instance", "batch_instance_device", "CONFIGS",
]


def rng_for(cfg: int, instance: int = 0, *extra: int) -> np.random.Generator:
    """Generator for config `cfg`, instance `instance` (plus optional sub-keys)."""
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, int(cfg), int(instance), *map(int, extra)]))


def logspace_to(count: int, top: float) -> np.ndarray:
    """Values 10^(alpha (i-1)), i = 1..count, alpha = log10(top)/(count-1): 1 .. top (Section 7)."""
    if count == 1:
        return np.ones(1)
    alpha = math.log10(top) / (count - 1)
    return 10.0 ** (alpha * np.arange(count, dtype=np.float64))


def haar(rng: np.random.Generator, m: int, n: Optional[int] = None) -> np.ndarray:
    """m x n matrix with Haar-distributed orthonormal columns (QR of a Gaussian, sign-fixed)."""
    n = m if n is None else n
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g)
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn


@dataclasses.dataclass
class Butterfly:
    """Random orthogonal V = P_r B_{r-1} P_{r-1} ... B_0 P_0 (P permutations, B block-diagonal Haar)."""

    m: int
    perms: list          # rounds + 1 permutations of range(m)
    blocks: list         # rounds lists of (start, stop, Haar block)

    def apply(self, x: np.ndarray) -> np.ndarray:
        """Return V @ x for x of shape (m, k) (x is not modified)."""
        y = np.ascontiguousarray(x[self.perms[0]])
        for r, blks in enumerate(self.blocks):
            for (s, e, b) in blks:
                y[s:e] = b @ y[s:e]
            y = np.ascontiguousarray(y[self.perms[r + 1]])
        return y

    def dense(self) -> np.ndarray:
        return self.apply(np.eye(self.m))

    def apply_torch(self, x):
        """V @ x for a torch tensor x of shape (m, k) on any device (same V as `apply`)."""
        import torch
        dev = x.device
        y = x.index_select(0, torch.as_tensor(self.perms[0], device=dev))
        for r, blks in enumerate(self.blocks):
            full = [b for b in blks if b[1] - b[0] == blks[0][1] - blks[0][0]]
            bs = full[0][1] - full[0][0]
            nf = len(full)
            stack = torch.as_tensor(np.stack([b[2] for b in full]), device=dev, dtype=y.dtype)
            head = y[: nf * bs].reshape(nf, bs, -1)
            y_new = torch.empty_like(y)
            y_new[: nf * bs] = torch.bmm(stack, head).reshape(nf * bs, -1)
            del head
            for (s_, e_, b) in blks[nf:]:
                y_new[s_:e_] = torch.as_tensor(b, device=dev, dtype=y.dtype) @ y[s_:e_]
            del y
            y = y_new.index_select(0, torch.as_tensor(self.perms[r + 1], device=dev))
            del y_new
        return y


def butterfly(rng: np.random.Generator, m: int, block: int = 256, rounds: int = 3) -> Butterfly:
    perms = [rng.permutation(m) for _ in range(rounds + 1)]
    blocks = []
    for _ in range(rounds):
        blks = []
        for s in range(0, m, block):
            e = min(m, s + block)
            blks.append((s, e, haar(rng, e - s)))
        blocks.append(blks)
    return Butterfly(m, perms, blocks)


def _symmetrize_inplace(a: np.ndarray, tile: int = 2048) -> None:
    m = a.shape[0]
    for i in range(0, m, tile):
        ie = min(m, i + tile)
        d = a[i:ie, i:ie]
        d[...] = 0.5 * (d + d.T)
        for j in range(ie, m, tile):
            je = min(m, j + tile)
            s = 0.5 * (a[i:ie, j:je] + a[j:je, i:ie].T)
            a[i:ie, j:je] = s
            a[j:je, i:ie] = s.T


def spd_from_eigs(v, d: np.ndarray) -> np.ndarray:
    """A = V diag(d) V^T, stored symmetric to the last bit (C order; equal to its transpose)."""
    if isinstance(v, Butterfly):
        m = v.m
        y = v.apply(np.diag(d))            # V D
        yt = np.ascontiguousarray(y.T)     # D V^T
        del y
        a = v.apply(yt)                    # V D V^T
        del yt
    else:
        a = (v * d) @ v.T
    _symmetrize_inplace(a)
    return a


def spd_from_eigs_torch(v: Butterfly, d: np.ndarray, device):
    """A = V diag(d) V^T for a Butterfly V, built with torch on `device` and stored exactly
    symmetric (same recipe as `spd_from_eigs`; rounding of the products may differ)."""
    import torch
    m = v.m
    y = torch.diag(torch.as_tensor(d, dtype=torch.float64, device=device))
    y = v.apply_torch(y)                       # V D
    y = v.apply_torch(y.t().contiguous())      # V D V^T
    a = y
    tile = 4096
    for i in range(0, m, tile):                # symmetrise in place, tile by tile
        ie = min(m, i + tile)
        a[i:ie, i:ie] = 0.5 * (a[i:ie, i:ie] + a[i:ie, i:ie].t())
        for j in range(ie, m, tile):
            je = min(m, j + tile)
            s_ = 0.5 * (a[i:ie, j:je] + a[j:je, i:ie].t())
            a[i:ie, j:je] = s_
            a[j:je, i:ie] = s_.t()
    return a


def dense_spd(rng: np.random.Generator, m: int, kappa: float, kind: str = "haar", block: int = 256):
    """Dense SPD A with eigenvalues logspace_to(m, kappa) and eigenvectors V.

    Returns (A, V, d) where V is an ndarray (kind="haar") or a Butterfly."""
    d = logspace_to(m, kappa)
    if kind == "haar":
        v = haar(rng, m)
    elif kind == "butterfly":
        v = butterfly(rng, m, block=block)
    else:
        raise ValueError(kind)
    return spd_from_eigs(v, d), v, d


def dense_spd_device(rng: np.random.Generator, m: int, kappa: float, device, block: int = 256):
    """Butterfly-eigenvector SPD A built on a torch device (for sizes where the host is too slow)."""
    d = logspace_to(m, kappa)
    v = butterfly(rng, m, block=block)
    return spd_from_eigs_torch(v, d, device), v, d


def tall_skinny(rng: np.random.Generator, m: int, n: int, kappa_z: float, u: Optional[np.ndarray] = None) -> np.ndarray:
    """Z = U diag(s) W^T with s = logspace_to(n, kappa_z) (descending) and Haar W.

    U defaults to a Haar m x n factor; its j-th column carries the j-th largest
    singular value.  Returned in Fortran (column-major) order."""
    if u is None:
        u = haar(rng, m, n)
    s = logspace_to(n, kappa_z)[::-1]
    w = haar(rng, n)
    return np.asfortranarray((u * s) @ w.T)


def gaussian_scaled(rng: np.random.Generator, m: int, n: int, kappa_z: float) -> np.ndarray:
    """Gaussian columns scaled by logspace_to(n, kappa_z), column-major."""
    g = np.asfortranarray(rng.standard_normal((n, m)).T)
    g *= logspace_to(n, kappa_z)
    return g


def paper_case(case: int, rng: np.random.Generator, m: int, n: int, kappa_a: float, kappa_z: float,
               v: Optional[np.ndarray] = None):
    """Test Cases 1-5 of Section 7.  Returns (A, Z, V, d).

    Eigenvalues ascend with the index (d_1 = 1, d_m = kappa(A)); within each
    case the largest singular value of Z pairs with the largest chosen
    eigenvalue.
      1: the n smallest eigenvalues;  2: the n largest;
      3: ceil(n/2) smallest and floor(n/2) largest;  4: random U;
      5: the eigenvectors of case 3 with singular values d^(-1/2) (Z is A-orthogonal).
    """
    d = logspace_to(m, kappa_a)
    if v is None:
        v = haar(rng, m)
    a = spd_from_eigs(v, d)
    lo, hi = (n + 1) // 2, n // 2
    if case == 1:
        idx = np.arange(n)
    elif case == 2:
        idx = np.arange(m - n, m)
    elif case in (3, 5):
        idx = np.concatenate([np.arange(lo), np.arange(m - hi, m)])
    elif case == 4:
        idx = None
    else:
        raise ValueError(case)
    if case == 4:
        z = tall_skinny(rng, m, n, kappa_z)
    elif case == 5:
        idx = idx[::-1]
        w = haar(rng, n)
        z = np.asfortranarray((v[:, idx] * d[idx] ** -0.5) @ w.T)
    else:
        idx = idx[::-1]                       # descending eigenvalue <-> descending singular value
        z = tall_skinny(rng, m, n, kappa_z, u=v[:, idx])
    return a, z, v, d


@dataclasses.dataclass(frozen=True)
class Stencil7:
    """Matrix-free 7-point operator on an nx x ny x nz grid, index p = x + nx (y + ny z).

    (A z)_p = center z_p + off * (sum of z over the in-grid face neighbours of p)
    (homogeneous Dirichlet boundary: neighbours outside the grid contribute 0)."""

    nx: int
    ny: int
    nz: int
    center: float
    off: float

    @property
    def m(self) -> int:
        return self.nx * self.ny * self.nz


def laplacian7(nx: int, ny: int, nz: int, shift: float = 1e-3) -> Stencil7:
    """Dirichlet 7-point Laplacian (h = 1) plus shift * I."""
    return Stencil7(nx, ny, nz, 6.0 + shift, -1.0)


@dataclasses.dataclass(frozen=True, eq=False)
class Tridiag:
    """Symmetric tridiagonal operator: A(i, i) = diag[i], A(i, i+1) = A(i+1, i) = sub[i]."""

    diag: np.ndarray
    sub: np.ndarray

    @property
    def m(self) -> int:
        return int(self.diag.shape[0])


def laplacian1d(m: int, shift: float = 1e-3) -> Tridiag:
    """Dirichlet 1D Laplacian (h = 1) plus shift * I: diagonal 2 + shift, off-diagonal -1."""
    return Tridiag(np.full(m, 2.0 + shift), np.full(max(m - 1, 0), -1.0))


@dataclasses.dataclass(frozen=True)
class BatchInstance:
    index: int
    m: int
    n: int
    kappa: float


def batch_plan(count: int = 4096, m_lo: int = 256, m_hi: int = 4096, n_set: Iterable[int] = (8, 16, 32, 64),
               k_lo: float = 1e2, k_hi: float = 1e8, cfg: int = 5) -> list:
    """Sizes of a batch: m log-uniform in [m_lo, m_hi], n uniform in n_set, kappa log-uniform."""
    rng = rng_for(cfg, 0)
    n_set = np.asarray(tuple(n_set))
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count))).astype(np.int64)
    ns = n_set[rng.integers(0, len(n_set), count)]
    ks = 10.0 ** rng.uniform(math.log10(k_lo), math.log10(k_hi), count)
    return [BatchInstance(i, int(ms[i]), int(ns[i]), float(ks[i])) for i in range(count)]


def batch_instance(inst: BatchInstance, dtype=np.float64, cfg: int = 5, block: int = 64):
    """(A_i, Z_i) of a batch instance: butterfly-Haar eigenvectors, Gaussian Z, rounded to dtype."""
    rng = rng_for(cfg, inst.index + 1)
    v = butterfly(rng, inst.m, block=block)
    a = spd_from_eigs(v, logspace_to(inst.m, inst.kappa))
    z = np.asfortranarray(rng.standard_normal((inst.n, inst.m)).T)
    return a.astype(dtype), z.astype(dtype)


def batch_instance_device(inst: BatchInstance, device, dtype=None, cfg: int = 5, block: int = 64):
    """`batch_instance` built with torch on `device`: A_i (m x m, contiguous, exactly symmetric) and
    Z_i as a column-major (m x n) view.  Same random draws as `batch_instance`; the products that
    form A_i round differently."""
    import torch
    dtype = dtype or torch.float64
    rng = rng_for(cfg, inst.index + 1)
    v = butterfly(rng, inst.m, block=block)
    a = spd_from_eigs_torch(v, logspace_to(inst.m, inst.kappa), device)
    z = torch.as_tensor(rng.standard_normal((inst.n, inst.m)), device=device)
    return a.to(dtype), z.to(dtype).t()


# The five workloads (sizes and spectra); generators above turn them into arrays.
CONFIGS = {
    1: dict(kind="dense", m=500, n=20, kappa_a=1e4, kappa_z=1e3, v="haar"),
    2: dict(kind="dense", m=8192, n=64, kappa_a=1e6, kappa_z=(1e1, 1e4, 1e7), v="haar"),
    3: dict(kind="stencil", grid=(128, 128, 64), shift=1e-3, n=128, kappa_z=1e4),
    4: dict(kind="dense", m=32768, n=256, kappa_a=1e8, kappa_z=1e5, v="butterfly"),
    5: dict(kind="batch", count=4096, m=(256, 4096), n=(8, 16, 32, 64), kappa=(1e2, 1e8)),
}
