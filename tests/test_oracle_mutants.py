"""Planted mistakes in copies of oracle routines must fail the pins (CPU only).

Each mutant is a plausible slip: the misprinted last line of the CHOL-EQR
listing (Q = C \\ Z), a transposed operand, a dropped sign fix, a dropped
stencil direction, a dropped operator in the Gram matrix, a wrong sign in a
Gram-Schmidt update.  The pin used is one of those in test_oracle_pins.
"""
import numpy as np
import scipy.linalg

import workloads as W
from oracle import exact, metrics, reference, stencil, variants

U = 2.0 ** -53


def _case():
    rng = W.rng_for(90, 3)
    a, _, _ = W.dense_spd(rng, 32, 1e4)
    z = W.tall_skinny(rng, 32, 5, 1e3)
    return a, z


def _pin_exact(f):
    a, z = _case()
    qe, re = exact.exact_oblique_qr(a, z)
    q, r = f(a, z)
    ok_r = metrics.r_forward_error(r, re) <= 50 * 32 * 5 * U * np.linalg.cond(re)
    ok_q = np.linalg.norm(q - qe) / np.linalg.norm(qe) <= 1e-9
    return ok_r and ok_q


def test_pin_accepts_the_real_oracle():
    assert _pin_exact(reference.chol_eqr)


def test_listing_misprint_q_equals_c_backslash_z_is_caught():
    def mutant(a, z):
        c = np.linalg.cholesky(a).T
        y, r = reference.householder_qr(c @ z)
        return scipy.linalg.solve_triangular(c, z, lower=False), r
    assert not _pin_exact(mutant)


def test_transposed_cholesky_factor_is_caught():
    def mutant(a, z):
        c = np.linalg.cholesky(a)              # lower used where the upper factor belongs
        y, r = reference.householder_qr(c @ z)
        return scipy.linalg.solve_triangular(c, y, lower=True), r
    assert not _pin_exact(mutant)


def test_missing_sign_fix_is_caught():
    def mutant(a, z):
        c = np.linalg.cholesky(a).T
        y, r = np.linalg.qr(c @ z)
        return scipy.linalg.solve_triangular(c, y, lower=False), r
    assert not _pin_exact(mutant)


def test_gram_without_operator_is_caught():
    def mutant(a, z):
        c = z.T @ z                            # A dropped from Z^T A Z
        r = np.linalg.cholesky(c).T
        return variants.trsm_right_upper(z, r), r
    assert not _pin_exact(mutant)


def test_cgs_sign_error_is_caught():
    def mutant(a, z):
        m, n = z.shape
        q = np.zeros((m, n)); r = np.zeros((n, n))
        for j in range(n):
            v = z[:, j].copy()
            if j:
                r[:j, j] = q[:, :j].T @ (a @ z[:, j])
                v = v + q[:, :j] @ r[:j, j]
            r[j, j] = np.sqrt(v @ a @ v)
            q[:, j] = v / r[j, j]
        return q, r
    assert _pin_exact(variants.cgs)
    assert not _pin_exact(mutant)


def test_stencil_dropped_direction_is_caught():
    st = W.laplacian7(5, 4, 3)
    ad = stencil.dense(st)
    x = W.rng_for(98).standard_normal((st.m, 2))

    def mutant(st_, x_):
        out = np.empty_like(x_)
        for j in range(x_.shape[1]):
            c = x_[:, j].reshape(st_.nz, st_.ny, st_.nx)
            y = st_.center * c
            y[:, :, 1:] += st_.off * c[:, :, :-1]
            y[:, :, :-1] += st_.off * c[:, :, 1:]
            y[:, 1:, :] += st_.off * c[:, :-1, :]
            y[:, :-1, :] += st_.off * c[:, 1:, :]
            out[:, j] = y.ravel()                 # z neighbours forgotten
        return out
    assert np.abs(stencil.apply(st, x) - ad @ x).max() < 1e-13
    assert np.abs(mutant(st, x) - ad @ x).max() > 0.1
