"""Pins for the CPU oracle: closed forms, brute force and theorems of the paper.

Nothing here compares the oracle with itself: every check is against exact
50-digit arithmetic, a closed form the paper's construction fixes (Section 7
Cases 1-5), Theorem 1.1, an independent algorithm, or a library routine that the
oracle does not use for that step.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact, metrics, mixed, reference, stencil, tridiag, variants

U = 2.0 ** -53


def tiny(seed, m=14, n=4, ka=1e3, kz=1e2):
    rng = W.rng_for(90, seed)
    a, _, _ = W.dense_spd(rng, m, ka)
    z = W.tall_skinny(rng, m, n, kz)
    return a, z


# ---- 1. exact arithmetic ---------------------------------------------------------------------

@pytest.mark.parametrize("seed,m,n", [(0, 8, 3), (1, 14, 4), (2, 20, 6), (3, 32, 5), (4, 9, 1)])
def test_chol_eqr_matches_50_digit_definition(seed, m, n):
    """Section 1: R = chol(Z^T A Z), Q = Z R^{-1}, evaluated at 50 digits."""
    a, z = tiny(seed, m, n, ka=1e4, kz=1e3)
    qe, re = exact.exact_oblique_qr(a, z)
    q, r = reference.chol_eqr(a, z)
    kap = np.linalg.cond(re)
    assert metrics.r_forward_error(r, re) <= 50 * m * n * U * kap
    assert np.linalg.norm(q - qe) / np.linalg.norm(qe) <= 50 * m * n * U * kap * np.linalg.cond(a) ** 0.5


def test_eqr_syev_matches_50_digit_definition():
    a, z = tiny(7, 16, 4, ka=1e3, kz=10)
    qe, re = exact.exact_oblique_qr(a, z)
    q, r = reference.eqr_syev(a, z)
    assert metrics.r_forward_error(r, re) < 1e-12
    assert np.abs(q - qe).max() / np.abs(qe).max() < 1e-11


def test_identity_inner_product_is_euclidean_qr():
    """A = I gives the Euclidean QR (Section 1); checked against 50-digit Gram-Schmidt-free
    definition and against CGS2, which shares no step with the oracle."""
    rng = W.rng_for(91)
    z = W.tall_skinny(rng, 24, 5, 1e3)
    a = np.eye(24)
    qe, re = exact.exact_oblique_qr(a, z)
    q, r = reference.chol_eqr(a, z)
    assert metrics.r_forward_error(r, re) < 1e-12
    assert np.abs(q.T @ q - np.eye(5)).max() < 1e-14
    q2, r2 = variants.cgs2(a, z)
    assert metrics.r_forward_error(r2, r) < 1e-12


def test_n_equals_one_closed_form():
    """n = 1: R = sqrt(z^T A z), Q = z / R."""
    rng = W.rng_for(92)
    a, _, _ = W.dense_spd(rng, 40, 1e5)
    z = rng.standard_normal((40, 1))
    q, r = reference.chol_eqr(a, z)
    zaz = math.fsum(float(z[i, 0]) * math.fsum(float(a[i, j]) * float(z[j, 0]) for j in range(40)) for i in range(40))
    assert abs(r[0, 0] - math.sqrt(zaz)) <= 1e-13 * math.sqrt(zaz)
    assert np.abs(q[:, 0] - z[:, 0] / math.sqrt(zaz)).max() <= 1e-12 * np.abs(z).max() / math.sqrt(zaz)


def test_diagonal_a():
    """A = D diagonal: Q = D^{-1/2} Y with [Y, R] = qr(D^{1/2} Z) (Section 1, B = D^{1/2})."""
    rng = W.rng_for(93)
    d = W.logspace_to(30, 1e6)
    z = W.tall_skinny(rng, 30, 5, 1e2)
    qe, re = exact.exact_oblique_qr(np.diag(d), z)
    q, r = reference.chol_eqr(np.diag(d), z)
    assert metrics.r_forward_error(r, re) < 1e-12
    assert np.abs(q - qe).max() / np.abs(qe).max() < 1e-11


# ---- 2. closed forms from the Section 7 constructions ----------------------------------------

def test_case5_gives_identity_r():
    """Case 5: Z = V_S D_S^{-1/2} W^T is A-orthogonal, so R = I and Q = Z."""
    rng = W.rng_for(94)
    a, z, v, d = W.paper_case(5, rng, 80, 10, 1e6, 1e3)
    q, r = reference.chol_eqr(a, z)
    # The computed A differs from V D V^T by O(u ||A||); the factor inherits O(u ||A|| ||Z||^2).
    tol = 100 * U * np.linalg.norm(a, 2) * np.linalg.norm(z, 2) ** 2
    assert np.abs(r - np.eye(10)).max() < tol
    assert np.abs(q - z).max() < tol * np.abs(z).max()


@pytest.mark.parametrize("case", [1, 2, 3])
def test_cases_1_to_3_singular_values_of_r(case):
    """Cases 1-3: Z = V_S Sigma W^T => sigma(R) = sorted{sqrt(d_j) s_j} (Theorem 1.1)."""
    rng = W.rng_for(95, case)
    m, n = 80, 10
    a, z, v, d = W.paper_case(case, rng, m, n, 1e6, 1e3)
    q, r = reference.chol_eqr(a, z)
    lo, hi = (n + 1) // 2, n // 2
    idx = {1: np.arange(n), 2: np.arange(m - n, m),
           3: np.concatenate([np.arange(lo), np.arange(m - hi, m)])}[case][::-1]
    s = W.logspace_to(n, 1e3)[::-1]
    expect = np.sort(np.sqrt(d[idx]) * s)[::-1]
    got = np.linalg.svd(r, compute_uv=False)
    kap = expect[0] / expect[-1]
    assert np.abs(got - expect).max() / expect[0] < 100 * U * kap


def test_theorem_1_1_on_random_input():
    """sigma_i(R) = sigma_i(A^{1/2} Z); ||Q||_2 = 1/sigma_n(A^{1/2} Zhat), A^{1/2} from eigh."""
    rng = W.rng_for(96)
    a, _, _ = W.dense_spd(rng, 120, 1e6)
    z = W.tall_skinny(rng, 120, 12, 1e4)
    q, r = reference.chol_eqr(a, z)
    lam, vv = np.linalg.eigh(a)
    ah = (vv * np.sqrt(lam)) @ vv.T
    s_expect = np.linalg.svd(ah @ z, compute_uv=False)
    s_got = np.linalg.svd(r, compute_uv=False)
    assert np.abs(s_got - s_expect).max() / s_expect[0] < 1e-11
    uz = np.linalg.svd(z, full_matrices=False)[0]
    sig = np.linalg.svd(ah @ uz, compute_uv=False)
    assert abs(np.linalg.norm(q, 2) - 1 / sig[-1]) < 1e-10 / sig[-1]
    sq = np.linalg.svd(q, compute_uv=False)
    assert np.allclose(sq, 1 / sig[::-1], rtol=1e-9)


# ---- 3. invariants and uniqueness ----------------------------------------------------------

def test_invariants_config1():
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    q, r = reference.chol_eqr(a, z)
    assert np.all(np.diag(r) > 0)
    assert np.all(np.tril(r, -1) == 0)
    assert metrics.orth_loss_dd(a, q) < 1e-13
    assert metrics.residual_f(z, q, r) < 1e-14
    for k in (1, 7, 20):   # nested spans: Z[:, :k] = Q[:, :k] R[:k, :k]
        assert np.linalg.norm(z[:, :k] - q[:, :k] @ r[:k, :k]) < 1e-13 * np.linalg.norm(z[:, :k])


def test_uniqueness_across_independent_routes():
    """Four routes with no common step give the same R (positive diagonal)."""
    rng = W.rng_for(97)
    a, _, _ = W.dense_spd(rng, 200, 1e4)
    z = W.tall_skinny(rng, 200, 8, 1e2)
    r0 = reference.chol_eqr(a, z)[1]
    kap = np.linalg.cond(r0)
    for f in (reference.eqr_syev, variants.cgs2, variants.cholqr2, variants.pre_cholqr):
        r = f(a, z)[1]
        assert metrics.r_forward_error(r, r0) < 100 * U * kap * 200, f.__name__


@pytest.mark.parametrize("seed,m,n", [(0, 8, 3), (1, 14, 4), (3, 32, 5)])
def test_upper_triangle_gram_matches_50_digit_definition(seed, m, n):
    """Algorithm 1 with the listing's chol(C) reading the upper triangle of C = Z^T (A Z): one pass
    within u kappa(R)^2 of the exact factor, two passes within u kappa(R)."""
    a, z = tiny(seed, m, n, ka=1e3, kz=1e2)
    qe, re = exact.exact_oblique_qr(a, z)
    kap = np.linalg.cond(re)
    r1 = variants.cholqr(a, z, gram="upper")[1]
    assert metrics.r_forward_error(r1, re) <= 50 * m * n * U * kap ** 2
    r2 = variants.cholqr2(a, z, gram="upper")[1]
    assert metrics.r_forward_error(r2, re) <= 50 * m * n * U * kap


def test_gram_conventions_agree_when_the_gram_is_exact():
    """Small integers: every product and sum is exact, so C is exactly symmetric and both readings of
    chol(C) factor the same matrix, bit for bit; R^T R reproduces Z^T A Z."""
    rng = np.random.default_rng(5)
    b = rng.integers(-3, 4, size=(12, 12)).astype(np.float64)
    a = b.T @ b + 12 * np.eye(12)
    z = rng.integers(-2, 3, size=(12, 4)).astype(np.float64)
    rs = variants.cholqr(a, z, gram="sym")[1]
    ru = variants.cholqr(a, z, gram="upper")[1]
    assert np.array_equal(rs, ru)
    assert np.allclose(ru.T @ ru, z.T @ a @ z, rtol=1e-14, atol=0)
    with pytest.raises(ValueError):
        variants.cholqr(a, z, gram="lower")


def _exact_zt_a_z(a, z):
    """Z^T A Z by brute-force integer sums (inputs hold small integers)."""
    ai, zi = a.astype(np.int64), z.astype(np.int64)
    m, n = zi.shape
    return np.array([[sum(int(zi[k, i]) * int(ai[k, l]) * int(zi[l, j]) for k in range(m) for l in range(m))
                      for j in range(n)] for i in range(n)], dtype=np.float64)


def test_split_gram_is_z_t_a_z_exactly_on_integers():
    """A = T + T^T with T = triu(A, 1) + diag(A)/2: on small integers every product and sum is exact,
    so the split assembly equals the integer Z^T A Z, and a T that keeps the whole diagonal (a
    plausible slip) does not."""
    rng = np.random.default_rng(11)
    b = rng.integers(-3, 4, size=(10, 10)).astype(np.float64)
    a = b.T @ b + 5 * np.eye(10)
    z = rng.integers(-2, 3, size=(10, 3)).astype(np.float64)
    exact_c = _exact_zt_a_z(a, z)
    assert np.array_equal(variants.split_gram(a, z), exact_c)
    t_bad = np.triu(a)                                 # planted slip: whole diagonal in T
    w = t_bad @ z
    assert not np.array_equal(z.T @ w + w.T @ z, exact_c)


def test_split_gram_is_exactly_symmetric_and_factors_within_theorem_bound():
    """The split assembly is symmetric by construction (M + M^T, bit for bit), and one CHOLQR pass on it
    lands within u kappa(R)^2 of the 50-digit factor, like the other readings of chol(C)."""
    a, z = tiny(1, 14, 4, ka=1e3, kz=1e2)
    c = variants.split_gram(a, z)
    assert np.array_equal(c, c.T)
    qe, re = exact.exact_oblique_qr(a, z)
    kap = np.linalg.cond(re)
    r1 = variants.cholqr(a, z, gram="split")[1]
    assert metrics.r_forward_error(r1, re) <= 50 * 14 * 4 * U * kap ** 2
    r2 = variants.cholqr2(a, z, gram="split")[1]
    assert metrics.r_forward_error(r2, re) <= 50 * 14 * 4 * U * kap


# ---- the tridiagonal operator (Section 8's sparse workload) ----------------------------------

def test_tridiag_apply_matches_assembled_matrix():
    rng = np.random.default_rng(8)
    t = W.Tridiag(rng.uniform(3, 4, 30), rng.uniform(-1, 1, 29))
    x = rng.standard_normal((30, 3))
    assert np.allclose(tridiag.apply(t, x), tridiag.dense(t) @ x, rtol=0, atol=1e-14)
    assert np.allclose(tridiag.apply(t, x[:, 0]), tridiag.dense(t) @ x[:, 0], rtol=0, atol=1e-14)


def test_laplacian1d_eigenvalues_closed_form():
    """Constant diagonal d and off-diagonal e: eigenvalues d + 2 e cos(pi k / (m + 1)), k = 1..m."""
    t = W.laplacian1d(50, shift=1e-2)
    lam = np.sort(2.01 - 2.0 * np.cos(np.pi * np.arange(1, 51) / 51))
    assert np.allclose(np.linalg.eigvalsh(tridiag.dense(t)), lam, rtol=1e-13, atol=1e-14)


def test_tridiag_eqr_matches_dense_route():
    """The banded CHOL-EQR (bidiagonal factor, banded solve) against the dense CHOL-EQR."""
    t = W.laplacian1d(200, shift=1e-2)
    z = W.tall_skinny(W.rng_for(94), 200, 6, 1e2)
    q, r = reference.tridiag_eqr(t, z)
    q0, r0 = reference.chol_eqr(tridiag.dense(t), z)
    kap = np.linalg.cond(r0)
    assert metrics.r_forward_error(r, r0) <= 100 * 6 * U * kap
    assert np.abs(q - q0).max() <= 100 * 6 * U * kap * np.abs(q0).max() * 20
    assert metrics.orth_loss(t, q) <= 1e-13


def test_gls_tridiag_matches_dense():
    t = W.laplacian1d(60, shift=1e-1)
    rng = np.random.default_rng(9)
    z = rng.standard_normal((60, 5))
    b = rng.standard_normal(60)
    assert np.allclose(reference.gls(t, z, b), reference.gls(tridiag.dense(t), z, b), rtol=1e-10, atol=0)


# ---- generalised least squares (Section 1) --------------------------------------------------

def test_gls_exact_when_b_is_in_the_range_of_z():
    a, z = tiny(11, 30, 5, ka=1e3, kz=1e2)
    xs = np.arange(1.0, 6.0)
    x = reference.gls(a, z, z @ xs)
    assert np.abs(x - xs).max() <= 100 * U * np.linalg.cond(z) * np.abs(xs).max()


def test_gls_satisfies_the_normal_equations():
    """Z^T A (Z x - b) = 0 (the A-orthogonality of the residual), and the definition's own formula
    R^{-1} Q^T A b with (Q, R) from the 50-digit oblique QR."""
    a, z = tiny(12, 24, 4, ka=1e4, kz=1e2)
    b = np.random.default_rng(3).standard_normal((24, 2))
    x = reference.gls(a, z, b)
    g = z.T @ a @ (z @ x - b)
    assert np.abs(g).max() <= 1e-9 * np.abs(z.T @ a @ b).max()
    qe, re = exact.exact_oblique_qr(a, z)
    xe = np.linalg.solve(re, qe.T @ a @ b)
    assert np.abs(x - xe).max() <= 1e-9 * np.abs(xe).max()


def test_gls_with_identity_is_ordinary_least_squares():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((40, 6))
    b = rng.standard_normal(40)
    x = reference.gls(np.eye(40), z, b)
    xo = np.linalg.pinv(z) @ b
    assert np.abs(x - xo).max() <= 1e-12 * np.abs(xo).max()


def test_gls_stencil_whitening_matches_dense():
    st = W.laplacian7(5, 4, 3)
    rng = np.random.default_rng(6)
    z = rng.standard_normal((st.m, 4))
    b = rng.standard_normal(st.m)
    x1 = reference.gls(st, z, b)
    x2 = reference.gls(stencil.dense(st), z, b)
    assert np.abs(x1 - x2).max() <= 1e-10 * np.abs(x2).max()


# ---- 4. the 7-point stencil ----------------------------------------------------------------

def test_stencil_apply_matches_assembled_matrix():
    st = W.laplacian7(5, 4, 3)
    ad = stencil.dense(st)
    assert np.array_equal(ad, ad.T)
    assert ad[0, 0] == st.center and ad[0, 1] == -1.0 and ad[0, 5] == -1.0 and ad[0, 20] == -1.0
    assert ad[4, 5] == 0.0            # x = 4 and x = 0 of the next row are not neighbours
    x = W.rng_for(98).standard_normal((st.m, 3))
    assert np.abs(stencil.apply(st, x) - ad @ x).max() < 1e-13


def test_stencil_eigenvalues_match_dense_eigensolver():
    st = W.laplacian7(6, 5, 4, shift=1e-3)
    lam = np.sort(stencil.eigenvalues(st).ravel())
    assert np.abs(lam - np.linalg.eigvalsh(stencil.dense(st))).max() < 1e-12
    big = W.laplacian7(128, 128, 64)
    assert abs(stencil.eigenvalues(big).min() - (1e-3 + 4 * (np.sin(np.pi / 258) ** 2 * 2 + np.sin(np.pi / 130) ** 2))) < 1e-15


def test_stencil_dst_route_matches_dense_route():
    st = W.laplacian7(7, 6, 5)
    z = W.gaussian_scaled(W.rng_for(99), st.m, 9, 1e4)
    qs, rs = reference.stencil_eqr(st, z)
    qd, rd = reference.chol_eqr(stencil.dense(st), z)
    assert metrics.r_forward_error(rs, rd) < 1e-14
    assert np.abs(qs - qd).max() / np.abs(qd).max() < 1e-13


# ---- 5. Cholesky with failure index -----------------------------------------------------

def test_chol_info_semantics():
    g = np.array([[4.0, 2, 0], [2, 5, 1], [0, 1, -3]])
    r, info = variants.chol_info(g)
    assert info == 3
    g2 = np.array([[4.0, 2], [2, 5]])
    r2, info2 = variants.chol_info(g2)
    assert info2 == 0 and np.allclose(r2.T @ r2, g2)
    g3 = np.array([[np.nan, 0], [0, 1.0]])
    assert variants.chol_info(g3)[1] == 1
    g4 = np.array([[1.0, 1], [1, 1]])        # singular: second pivot exactly zero
    assert variants.chol_info(g4)[1] == 2


# ---- 6. error-free check and the bfloat16 model -------------------------------------------------

def test_orth_loss_dd_against_50_digits():
    import mpmath
    a, z = tiny(11, 16, 4)
    q, r = reference.chol_eqr(a, z)
    with mpmath.workdps(50):
        Q = [[mpmath.mpf(float(v)) for v in row] for row in q]
        A = [[mpmath.mpf(float(v)) for v in row] for row in a]
        AQ = [[mpmath.fsum(A[i][k] * Q[k][j] for k in range(16)) for j in range(4)] for i in range(16)]
        E = np.array([[float(mpmath.fsum(Q[k][i] * AQ[k][j] for k in range(16)) - (1 if i == j else 0))
                       for j in range(4)] for i in range(4)])
    exact_loss = np.linalg.norm(E, 2)
    assert abs(metrics.orth_loss_dd(a, q) - exact_loss) <= 1e-3 * exact_loss + 1e-30


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = W.rng_for(100).standard_normal(10000) * 10.0 ** W.rng_for(101).uniform(-8, 8, 10000)
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mixed.bf16(x32), ref)


def test_bf16_split_representation_error():
    x = W.rng_for(102).standard_normal(10000)
    s2 = mixed.split(x, 2)
    s3 = mixed.split(x, 3)
    e2 = np.abs(x - s2[0] - s2[1]) / np.abs(x)
    e3 = np.abs(x - s3[0] - s3[1] - s3[2]) / np.abs(x)
    assert e2.max() <= 2.0 ** -16 * 1.01 and e3.max() <= 2.0 ** -24 * 1.01
