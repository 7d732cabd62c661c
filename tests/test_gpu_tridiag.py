"""GPU parity for the symmetric tridiagonal operator (the paper's sparse workload, Section 8): every
entry point that takes an operator, against the oracle's banded CHOL-EQR (Algorithm 3 with LAPACK
banded Cholesky and solve) on the same inputs.  Bars as for the dense paths: residual <= 1e-12,
orthogonality <= 1e-12 for the stable variants, R forward error <= 10 n u kappa(R)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev_colmajor, to_host
from oracle import metrics, reference, variants

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")


def case(m, n, shift=1e-3, kz=1e3, seed=0):
    t = W.laplacian1d(m, shift)
    z = W.tall_skinny(W.rng_for(95, seed, m, n), m, n, kz)
    return t, z


def op(t):
    return oqr.Tridiag(t.diag, t.sub)


def stable_checks(t, z, q, r, r0):
    n = z.shape[1]
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(t, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)


@pytest.mark.parametrize("pass1", ["fp64", "bf16x3"])
def test_tridiag_cholqr2(pass1):
    t, z = case(5003, 40)
    q0, r0 = reference.tridiag_eqr(t, z)
    banner(f"tridiag cholqr2 {pass1}")
    q, r = (to_host(x) for x in oqr.cholqr2(op(t), to_dev_colmajor(z), pass1=pass1))
    stable_checks(t, z, q, r, r0)


def test_tridiag_large_m():
    """m = 100000 (the paper's size): more than four 64-row tiles per CU, the persistent substitution."""
    t, z = case(100000, 16, seed=1)
    q0, r0 = reference.tridiag_eqr(t, z)
    banner("tridiag m=100000")
    A = op(t)
    Z = to_dev_colmajor(z)
    Q, R = oqr.cholqr2(A, Z)
    stable_checks(t, z, to_host(Q), to_host(R), r0)
    orth_f, res = oqr.check(A, Z, Q, R)
    assert orth_f <= 1e-12 and res <= 1e-12


def test_tridiag_chol_eqr():
    t, z = case(4000, 24, seed=2)
    q0, r0 = reference.tridiag_eqr(t, z)
    banner("tridiag chol_a")
    q, r = (to_host(x) for x in oqr.chol_a(op(t), to_dev_colmajor(z)))
    stable_checks(t, z, q, r, r0)
    assert np.abs(q - q0).max() <= 100 * 24 * U * np.linalg.cond(r0) * np.abs(q0).max() * 10


def test_tridiag_chol_eqr_large_m():
    """m = 100000: the pivot recurrence and the bidiagonal back-substitution run in chunks of rows
    (391 of them) joined by the chunk-to-chunk maps."""
    t, z = case(100000, 16, seed=5)
    q0, r0 = reference.tridiag_eqr(t, z)
    banner("tridiag chol_a m=100000")
    q, r = (to_host(x) for x in oqr.chol_a(op(t), to_dev_colmajor(z)))
    stable_checks(t, z, q, r, r0)
    assert np.abs(q - q0).max() <= 100 * 16 * U * np.linalg.cond(r0) * np.abs(q0).max() * 10


@pytest.mark.parametrize("m,bad", [(300, 150), (3000, 1000), (3000, 2999)])
def test_tridiag_chol_eqr_reports_the_failing_pivot(m, bad):
    d = np.full(m, 2.001)
    d[bad] = -1.0
    t = W.Tridiag(d, np.full(m - 1, -1.0))
    z = np.zeros((m, 3), order="F")
    z[0, 0] = z[1, 1] = z[2, 2] = 1.0
    plan = oqr.Plan("chol_a", op(t), 3)
    with pytest.raises(oqr.OQRError) as e:
        plan(to_dev_colmajor(z))
    from oracle import tridiag
    assert e.value.info == variants.chol_info(tridiag.dense(t))[1]


@pytest.mark.parametrize("alg", ["pre_cholqr", "cgs2"])
def test_tridiag_other_variants(alg):
    t, z = case(2000, 20, seed=3)
    q0, r0 = reference.tridiag_eqr(t, z)
    banner(f"tridiag {alg}")
    if alg == "cgs2":
        q, r = (to_host(x) for x in oqr.gs(op(t), to_dev_colmajor(z), variant="cgs2"))
    else:
        q, r = (to_host(x) for x in oqr.pre_cholqr(op(t), to_dev_colmajor(z)))
    stable_checks(t, z, q, r, r0)


def test_tridiag_gls():
    t, z = case(3000, 10, shift=1e-1, kz=1e2, seed=4)
    b = np.random.default_rng(25).standard_normal((3000, 2))
    A = op(t)
    Q, R = oqr.cholqr2(A, to_dev_colmajor(z))
    x = to_host(oqr.gls(A, Q, R, to_dev_colmajor(b)))
    x0 = reference.gls(t, z, b)
    kr = np.linalg.cond(to_host(R))
    assert np.abs(x - x0).max() <= 1e3 * 10 * U * kr * kr * np.abs(x0).max()


def test_tridiag_single_row():
    t = W.Tridiag(np.array([4.0]), np.zeros(0))
    z = np.array([[3.0]])
    q, r = (to_host(x) for x in oqr.cholqr2(op(t), to_dev_colmajor(z)))
    assert abs(r[0, 0] - 6.0) <= 4 * U * 6 and abs(q[0, 0] - 0.5) <= 4 * U


@pytest.mark.parametrize("m", [1, 2, 257, 512, 513])
def test_tridiag_chol_eqr_chunk_edges(m):
    """CHOL-EQR at sizes around the 256-row chunks of its recurrences (one row, a last chunk of one row,
    exact multiples)."""
    t = W.laplacian1d(m, 1e-1)
    n = min(m, 4)
    z = W.tall_skinny(W.rng_for(96, m), m, n, 10.0 if n > 1 else 1.0)
    q0, r0 = reference.tridiag_eqr(t, z)
    banner(f"tridiag chol_a m={m}")
    q, r = (to_host(x) for x in oqr.chol_a(op(t), to_dev_colmajor(z)))
    assert metrics.residual_f(z, q, r) <= 1e-13
    assert metrics.orth_loss(t, q) <= 1e-13
    assert metrics.r_forward_error(r, r0) <= 100 * n * U * np.linalg.cond(r0) * 10
