"""GPU parity of the baselines behind the same ABI: Gram-Schmidt in the A inner product (CGS,
MGS row/column oriented, CGS2; Section 6), CHOL-EQR (Algorithm 3) and EQR-SYEV (Algorithm 4).

Each GPU routine is compared with the oracle's FP64 implementation of the same algorithm on the
same seeded inputs.  Both are rounding-perturbed runs of one algorithm, so the bars are the
algorithm's own error model (stated per test), plus the properties every correct run has: the
residual ||Z - QR||_F / ||Z||_F <= 1e-12, R upper triangular with positive diagonal, and an
orthogonality loss within 10x (plus a floor) of the oracle's run of the same algorithm.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from oracle import metrics, reference, variants

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")

GS = ["cgs", "mgs_row", "mgs_col", "cgs2"]
ORACLE_GS = {"cgs": variants.cgs, "mgs_row": variants.mgs_row, "mgs_col": variants.mgs_col, "cgs2": variants.cgs2}


def dense_case(cfg, m, n, ka, kz, seed=0):
    rng = W.rng_for(cfg, seed, m, n)
    a, _, _ = W.dense_spd(rng, m, ka)
    z = W.tall_skinny(rng, m, n, kz)
    return a, z


def gpu(alg, A, z, **kw):
    q, r = getattr(oqr, alg)(A, to_dev_colmajor(z), **kw)
    return to_host(q), to_host(r)


def common_checks(a, z, q, r, q0, r0, orth_floor=1e-13):
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + orth_floor


# ---- Gram-Schmidt ------------------------------------------------------------------------------

@pytest.mark.parametrize("variant", GS)
def test_gs_well_conditioned_matches_oracle_elementwise(variant):
    """kappa(A^{1/2} Z) ~ 1e2: the R and Q of two FP64 runs agree to n u kappa^2 (CGS's bound)."""
    a, z = dense_case(61, 300, 24, 1e2, 1e1)
    q0, r0 = ORACLE_GS[variant](a, z)
    banner(f"gs {variant} well conditioned")
    q, r = gpu("gs", to_dev(a), z, variant=variant)
    kap = np.linalg.cond(r0)
    tol = 100 * z.shape[1] * U * kap ** 2
    assert metrics.r_forward_error(r, r0) <= tol
    assert np.abs(q - q0).max() <= tol * np.abs(q0).max()
    common_checks(a, z, q, r, q0, r0)


@pytest.mark.parametrize("variant", GS)
def test_gs_config1(variant):
    """m=500, n=20, kappa(A)=1e4, kappa(Z)=1e3: residual and orthogonality behave as the oracle's."""
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    q0, r0 = ORACLE_GS[variant](a, z)
    banner(f"gs {variant} config1")
    q, r = gpu("gs", to_dev(a), z, variant=variant)
    common_checks(a, z, q, r, q0, r0)
    if variant in ("mgs_row", "mgs_col", "cgs2"):
        # the stable-R variants: R forward error n u kappa(R) against CHOL-EQR's R
        _, rc = reference.chol_eqr(a, z)
        assert metrics.r_forward_error(r, rc) <= 100 * z.shape[1] * U * np.linalg.cond(rc)


@pytest.mark.parametrize("variant", ["cgs2", "mgs_row"])
def test_gs_larger_dense(variant):
    """A shape with several 1024-row chunks and a ragged tail: m=2500, n=40."""
    a, z = dense_case(62, 2500, 40, 1e6, 1e3)
    q0, r0 = ORACLE_GS[variant](a, z)
    banner(f"gs {variant} m=2500")
    q, r = gpu("gs", to_dev(a), z, variant=variant)
    common_checks(a, z, q, r, q0, r0)


@pytest.mark.parametrize("variant", GS)
def test_gs_stencil(variant):
    st = W.laplacian7(9, 8, 7)
    rng = W.rng_for(63, 0)
    z = W.tall_skinny(rng, st.m, 16, 1e2)
    q0, r0 = ORACLE_GS[variant](st, z)
    banner(f"gs {variant} stencil")
    q, r = gpu("gs", oqr.Stencil7(9, 8, 7, st.center, st.off), z, variant=variant)
    assert metrics.residual_f(z, q, r) <= 1e-12
    kap = np.linalg.cond(r0)
    assert metrics.r_forward_error(r, r0) <= 100 * z.shape[1] * U * kap ** 2
    from oracle import stencil
    g = q.T @ stencil.apply(st, q)
    g0 = q0.T @ stencil.apply(st, q0)
    assert np.linalg.norm(np.eye(16) - g, 2) <= 10 * np.linalg.norm(np.eye(16) - g0, 2) + 1e-13


@pytest.mark.parametrize("variant", GS)
def test_gs_single_column(variant):
    a, z = dense_case(64, 40, 1, 1e2, 1.0)
    q0, r0 = ORACLE_GS[variant](a, z)
    q, r = gpu("gs", to_dev(a), z, variant=variant)
    assert abs(r[0, 0] - r0[0, 0]) <= 10 * U * r0[0, 0]
    assert np.abs(q - q0).max() <= 10 * U * np.abs(q0).max()


def test_gs_reports_nonpositive_norm():
    """A indefinite on span(Z): the column whose A-norm^2 is <= 0 is reported (1-based)."""
    m, n = 64, 4
    d = np.ones(m)
    d[2] = -5.0
    a = np.diag(d)
    z = np.zeros((m, n), order="F")
    for j in range(n):
        z[j, j] = 1.0
    for variant in GS:
        plan = oqr.Plan("gs", to_dev(a), n, gs_variant=variant)
        with pytest.raises(oqr.OQRError) as e:
            plan(to_dev_colmajor(z))
        assert e.value.info == 3, variant


# ---- CHOL-EQR --------------------------------------------------------------------------------

def chol_eqr_tol(a, r0, n):
    # perturbations of C and of W = C Z are amplified by kappa(C) = kappa(A)^{1/2}, then by kappa(R)
    return 100 * n * U * np.sqrt(np.linalg.cond(a)) * np.linalg.cond(r0)


def test_chol_a_config1():
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    q0, r0 = reference.chol_eqr(a, z)
    banner("chol_a config1")
    q, r = gpu("chol_a", to_dev(a), z)
    common_checks(a, z, q, r, q0, r0)
    tol = chol_eqr_tol(a, r0, 20)
    assert metrics.r_forward_error(r, r0) <= tol
    assert np.abs(q - q0).max() <= tol * np.abs(q0).max()


@pytest.mark.parametrize("m,n", [(1, 1), (63, 5), (130, 64), (1100, 70)])
def test_chol_a_ragged(m, n):
    """Panels of 64 with ragged last panels, QR columns past one 64-column block."""
    a, z = dense_case(65, m, n, 1e3, 1e2)
    q0, r0 = reference.chol_eqr(a, z)
    banner(f"chol_a m={m} n={n}")
    q, r = gpu("chol_a", to_dev(a), z)
    common_checks(a, z, q, r, q0, r0)
    assert metrics.r_forward_error(r, r0) <= chol_eqr_tol(a, r0, n)


def test_chol_a_reports_first_failing_pivot():
    m, n = 150, 4
    rng = W.rng_for(66)
    a, _, _ = W.dense_spd(rng, m, 1e2)
    a[100, 100] = -1.0            # breaks positive definiteness at a pivot <= 101
    z = W.tall_skinny(rng, m, n, 1e1)
    want = variants.chol_info(a)[1]
    assert want > 0
    plan = oqr.Plan("chol_a", to_dev(a), n)
    with pytest.raises(oqr.OQRError) as e:
        plan(to_dev_colmajor(z))
    assert e.value.info == want


# ---- EQR-SYEV ----------------------------------------------------------------------------------

def eqr_syev_tol(a, r0, n):
    return 100 * n * U * np.linalg.cond(a) * np.linalg.cond(r0)


@pytest.mark.parametrize("m,n", [(2, 1), (9, 3), (301, 12)])
def test_eig_a_small_and_odd(m, n):
    """Odd m exercises the padding index of the round-robin ordering."""
    a, z = dense_case(67, m, n, 1e3, 1e2)
    q0, r0 = reference.eqr_syev(a, z)
    banner(f"eig_a m={m} n={n}")
    q, r = gpu("eig_a", to_dev(a), z)
    common_checks(a, z, q, r, q0, r0)
    assert metrics.r_forward_error(r, r0) <= eqr_syev_tol(a, r0, n)


def test_eig_a_config1():
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    q0, r0 = reference.eqr_syev(a, z)
    banner("eig_a config1")
    q, r = gpu("eig_a", to_dev(a), z)
    common_checks(a, z, q, r, q0, r0)
    tol = eqr_syev_tol(a, r0, 20)
    assert metrics.r_forward_error(r, r0) <= tol
    assert np.abs(q - q0).max() <= tol * np.abs(q0).max()


def test_eig_a_reports_nonpositive_eigenvalue():
    m, n = 40, 3
    rng = W.rng_for(68)
    v = W.haar(rng, m, m)
    d = np.linspace(1.0, 2.0, m)
    d[7] = -0.5
    a = W.spd_from_eigs(v, d)
    z = W.tall_skinny(rng, m, n, 1e1)
    plan = oqr.Plan("eig_a", to_dev(a), n)
    with pytest.raises(oqr.OQRError) as e:
        plan(to_dev_colmajor(z))
    assert e.value.info == 1


def test_baselines_reject_stencil_operator_for_dense_only_algorithms():
    st = W.laplacian7(4, 4, 4)
    z = np.zeros((st.m, 2), order="F")
    z[0, 0] = z[1, 1] = 1.0
    for alg in ("chol_a", "eig_a"):
        with pytest.raises(oqr.OQRError):
            getattr(oqr, alg)(oqr.Stencil7(4, 4, 4, st.center, st.off), to_dev_colmajor(z))
