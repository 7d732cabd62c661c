"""GPU parity of the FP32 operand pass (`pass1="fp32"`): the operator product (dense A) or the Gram
product (stencil and tridiagonal A, on W = A Z formed in FP64) with both operands rounded to FP32,
products on FP32 MFMA, FP32 sums inside a tile of K and FP64 across tiles; the Cholesky
factorisation (with the reduced-precision shift) and the substitution stay FP64.

Bars: one FP32 pass loses orthogonality at the level of the CPU emulation of the same arithmetic
(`oracle.mixed.cholqr_pass` with the FP32 scheme; within 10x: level, not bits, since the order of the
sums differs), and its residual stays at the FP64 level (the substitution is FP64, Theorem 2.1's
residual bound); followed by an FP64 pass (CholQR2-A) it reaches the stable level (<= 1e-12) where
the first pass's shift allows it, R within 10 n u kappa(R) of the oracle's; both passes FP32 reach
max(1e-6, 10 u32 ||A|| ||Q||^2).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from oracle import metrics, mixed, reference

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")

U32 = 2.0 ** -24


def dense_case(m, n, ka, kz, seed=0):
    rng = W.rng_for(11, seed, m, n)
    a, _, _ = W.dense_spd(rng, m, ka, kind="butterfly" if m > 2048 else "haar")
    z = W.tall_skinny(rng, m, n, kz)
    return a, z


def run(alg, A, z, **kw):
    q, r = getattr(oqr, alg)(A, to_dev_colmajor(z), **kw)
    return to_host(q), to_host(r)


@pytest.mark.parametrize("m,n", [(2048, 64), (1531, 129), (600, 256), (3000, 50)])
def test_dense_fp32_pass_at_emulated_level(m, n):
    a, z = dense_case(m, n, 1e4, 1e3, seed=m)
    qe, _, info, _ = mixed.cholqr_pass(a, z, "fp32", 1.0, 3, kt=960, symmetric_blocks=64)
    assert info == 0
    banner(f"fp32 pass dense m={m} n={n}")
    q, r = run("cholqr", to_dev(a), z, prec="fp32")
    le, lg = metrics.orth_loss(a, qe), metrics.orth_loss(a, q)
    assert le / 10 <= lg <= 10 * le, (le, lg)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)


@pytest.mark.parametrize("m,n,kz", [(2048, 64, 1e4), (777, 100, 1e5), (4096, 256, 1e3)])
def test_dense_fp32_then_fp64_reaches_fp64_orthogonality(m, n, kz):
    a, z = dense_case(m, n, 1e6, kz, seed=m + 1)
    _, r0 = reference.chol_eqr(a, z)
    banner(f"fp32+fp64 cholqr2 dense m={m} n={n}")
    q, r = run("cholqr2", to_dev(a), z, pass1="fp32", pass2="fp64")
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(a, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)


def test_dense_fully_fp32_cholqr2_meets_the_reduced_precision_bar():
    a, z = dense_case(1500, 40, 1e5, 1e3, seed=3)
    q0, r0 = reference.chol_eqr(a, z)
    aq2 = metrics.diagnostics(a, z, q0, r0)["a_q2"]
    banner("fp32+fp32 cholqr2 dense")
    q, r = run("cholqr2", to_dev(a), z, pass1="fp32", pass2="fp32")
    assert metrics.orth_loss(a, q) <= max(1e-6, 10 * U32 * aq2)
    assert metrics.residual_f(z, q, r) <= 1e-12


@pytest.mark.parametrize("grid,n", [((20, 24, 9), 100), ((32, 32, 16), 64), ((16, 12, 10), 150)])
def test_stencil_fp32_pass(grid, n):
    st = W.laplacian7(*grid)
    z = W.tall_skinny(W.rng_for(12, 0, *grid), st.m, n, 1e3)
    qe, _, info, _ = mixed.cholqr_pass(st, z, "fp32", 1.0, 3)
    assert info == 0
    op = oqr.Stencil7(*grid, st.center, st.off)
    banner(f"fp32 pass stencil grid={grid} n={n}")
    q, r = run("cholqr", op, z, prec="fp32")
    le, lg = metrics.orth_loss(st, qe), metrics.orth_loss(st, q)
    assert le / 10 <= lg <= 10 * le, (le, lg)
    assert metrics.residual_f(z, q, r) <= 1e-12
    banner(f"fp32+fp64 cholqr2 stencil grid={grid} n={n}")
    q2, r2 = run("cholqr2", op, z, pass1="fp32", pass2="fp64")
    _, r0 = reference.stencil_eqr(st, z)
    assert metrics.residual_f(z, q2, r2) <= 1e-12
    assert metrics.orth_loss(st, q2) <= 1e-12
    assert metrics.r_forward_error(r2, r0) <= 10 * n * U * np.linalg.cond(r0)


def test_stencil_fp64_then_fp32_second_pass():
    """An FP32 second pass after a fused FP64 first pass: the first-pass Q is not kept in the workspace
    that the unfused FP32 Gram uses for A Q1."""
    grid, n = (24, 20, 12), 48
    st = W.laplacian7(*grid)
    z = W.tall_skinny(W.rng_for(12, 1, *grid), st.m, n, 1e2)
    op = oqr.Stencil7(*grid, st.center, st.off)
    banner("fp64+fp32 cholqr2 stencil")
    q, r = run("cholqr2", op, z, pass1="fp64", pass2="fp32")
    q0, r0 = reference.stencil_eqr(st, z)
    aq2 = metrics.diagnostics(st, z, q0, r0)["a_q2"]
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= max(1e-6, 10 * U32 * aq2)


def test_tridiag_fp32_then_fp64():
    m, n = 20000, 32
    t = W.laplacian1d(m)
    z = W.tall_skinny(W.rng_for(12, 2), m, n, 1e3)
    A = oqr.Tridiag(t.diag, t.sub)
    banner("fp32+fp64 cholqr2 tridiagonal")
    q, r = run("cholqr2", A, z, pass1="fp32", pass2="fp64")
    _, r0 = reference.tridiag_eqr(t, z)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(t, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)
