"""The per-algorithm references against the error behaviour Section 7 reports.

m = 80, n = 10 as in the paper's experiments; kappa(Z) = kappa(A)^{1/2}.  Bands
are wide (the paper drops the constants of its bounds when plotting); what is
pinned is the scaling law, which a dropped term, a wrong index or a transposed
operand in a reference would break.
"""
import numpy as np
import pytest

import workloads as W
from oracle import metrics, reference, variants

U = 2.0 ** -53
M, N = 80, 10
STABLE = {
    "chol_eqr": reference.chol_eqr, "eqr_syev": reference.eqr_syev, "cgs2": variants.cgs2,
    "pre_cholqr": variants.pre_cholqr,
}
ALL = dict(STABLE, cholqr2=variants.cholqr2, cholqr=variants.cholqr, cgs=variants.cgs, mgs_row=variants.mgs_row, mgs_col=variants.mgs_col)


def run(case, ka, kz, seed=0):
    rng = W.rng_for(80, case, seed, int(np.log10(ka)))
    a, z, v, d = W.paper_case(case, rng, M, N, ka, kz)
    return a, z


@pytest.mark.parametrize("case", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("ka", [1e4, 1e10])
def test_stable_algorithms_loss_bounded_by_a_q2(case, ka):
    """Loss of the stable class is c u ||A|| ||Q||^2 (Theorems 3.1, 4.1, 5.1, 6.4)."""
    a, z = run(case, ka, ka ** 0.5)
    q0, r0 = reference.chol_eqr(a, z)
    aq2 = metrics.diagnostics(a, z, q0, r0)["a_q2"]
    for name, f in STABLE.items():
        q, r = f(a, z)
        assert metrics.orth_loss(a, q) <= 10 * M * N * U * aq2, name
    # CHOLQR twice joins the stable class once the first pass cannot break down
    # (Theorem 2.1 with Z = Q1, kappa(A^{1/2} Q1) ~ 1).
    if U * np.linalg.cond(r0) ** 2 < 1e-2:
        q, r = variants.cholqr2(a, z)
        assert metrics.orth_loss(a, q) <= 10 * M * N * U * aq2


def test_case1_reaches_kappa_a():
    """Cases 1, 3, 5 attain the worst case ||A|| ||Q||^2 = kappa(A)."""
    a, z = run(1, 1e12, 1e6)
    q, r = reference.chol_eqr(a, z)
    d = metrics.diagnostics(a, z, q, r)
    assert 0.3e12 < d["a_q2"] <= 1.01e12
    assert metrics.orth_loss(a, q) > 1e-3 * U * 1e12


def test_cholqr_and_cgs_lose_kappa_z_squared_in_case2():
    """Case 2: CHOLQR and CGS lose orthogonality like kappa(Z)^2, MGS like kappa(Z)."""
    lo = run(2, 1e4, 1e2)
    hi = run(2, 1e8, 1e4)
    for name, law in (("cholqr", 1e4), ("cgs", 1e4), ("mgs_row", 1e2), ("mgs_col", 1e2)):
        f = ALL[name]
        l0 = metrics.orth_loss(lo[0], f(*lo)[0])
        l1 = metrics.orth_loss(hi[0], f(*hi)[0])
        assert law / 30 < l1 / l0 < law * 30, (name, l0, l1)
    # and the stable class does not depend on kappa(Z) there
    l0 = metrics.orth_loss(lo[0], reference.chol_eqr(*lo)[0])
    l1 = metrics.orth_loss(hi[0], reference.chol_eqr(*hi)[0])
    assert l1 / l0 < 100


def test_case5_all_algorithms_alike():
    """Case 5 (Z A-orthogonal): every algorithm shows the same loss level."""
    a, z = run(5, 1e8, 1e4)
    losses = {k: metrics.orth_loss(a, f(a, z)[0]) for k, f in ALL.items()}
    vals = np.array(list(losses.values()))
    assert vals.max() / vals.min() < 100, losses


@pytest.mark.parametrize("case", [2, 3, 4])
def test_syev_residual_grows_with_sqrt_kappa_a(case):
    """EQR-SYEV representativity error grows like kappa(A)^{1/2} in Cases 2-4 (Theorem 5.1)."""
    res = []
    for ka in (1e4, 1e12):
        a, z = run(case, ka, 10.0)
        q, r = reference.eqr_syev(a, z)
        res.append(metrics.residual_2(z, q, r))
    assert 1e4 / 100 < res[1] / res[0] < 1e4 * 100, res


@pytest.mark.parametrize("case", [1, 2, 3, 4])
def test_representativity_constant_for_cholqr_and_gs(case):
    """CHOLQR, PRE-CHOLQR, CGS, MGS and CGS2 keep ~1e-15 relative residual (Section 7)."""
    for ka in (1e4, 1e12):
        a, z = run(case, ka, ka ** 0.5)
        for name in ("cholqr", "pre_cholqr", "cgs", "mgs_row", "mgs_col", "cgs2"):
            try:
                q, r = ALL[name](a, z)
            except np.linalg.LinAlgError:
                assert name == "cholqr" and ka == 1e12   # the Cholesky may break down (kappa^2 u > 1)
                continue
            assert metrics.residual_2(z, q, r) < 1e-13, (name, ka)


def test_chol_eqr_a_norm_residual():
    """Theorem 4.1 / Section 7 (kappa(Z) = 10): the A-norm residual of CHOL-EQR stays at
    rounding level in Cases 2-4 and grows like kappa(A)^{1/2} only in Case 1."""
    for case in (2, 3, 4):
        for ka in (1e4, 1e12):
            a, z = run(case, ka, 10.0)
            q, r = reference.chol_eqr(a, z)
            assert metrics.residual_a(a, z, q, r) < 1e-14
    res = []
    for ka in (1e4, 1e12):
        a, z = run(1, ka, 10.0)
        q, r = reference.chol_eqr(a, z)
        res.append(metrics.residual_a(a, z, q, r))
    assert 1e4 / 30 < res[1] / res[0] < 1e4 * 30, res
