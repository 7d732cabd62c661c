"""The dense FP64 workload at its stated size: m = 8192, n = 64, A = V diag(d) V^T with Haar V and d
log-spaced 1..1e6, Z = U diag(s) W^T (Haar U, W) with kappa(Z) in {1e1, 1e4, 1e7} (Section 7's test
matrices), every variant against the oracle's run of the same algorithm.

Bars (the error models of Sections 2-6):
* CholQR2-A with an FP64 first and second pass: residual and A-orthogonality <= 1e-12 (the stable
  class), R within 10 n u kappa(R) of CHOL-EQR's R (the unique factor).
* CholQR2-A with a split-bfloat16 first pass (bf16x2 or bf16x3) and an FP64 second: the first
  attempt of the reduced-precision pass adds s = 2^-24 max_i G_ii to the Gram (and its products
  carry errors of that order), which leaves kappa(A^{1/2} Q1) of order (2^-24)^{1/2} kappa(A^{1/2} Z);
  the FP64 second pass then ends at c u kappa(A^{1/2} Q1)^2 (Theorem 2.1 with Z = Q1): at
  kappa(Z) = 1e7 (kappa(A^{1/2} Z) about 1e7) that is about 1e-11, above 1e-12.  Bar: orthogonality
  <= max(1e-12, 10x the CPU emulation of the same schedule), residual <= 1e-12, R within
  10 n u kappa(R) + kappa(R) x (the orthogonality reached).
* CHOLQR-A, CGS-A, MGS-A (both orientations), CGS2-A, PRE-CHOLQR-A: residual <= 1e-12, R upper
  triangular with a positive diagonal, orthogonality within 10x (plus a floor) of the same algorithm
  on the CPU, and R within the algorithm's perturbation bound of the CPU run's R (u kappa(R)^2 for
  the Gram-based CHOLQR-A and CGS-A, whose computed Gram carries an error of u ||G||).
* CHOL-EQR: R and Q within 100 n u kappa(A)^{1/2} kappa(R) of the oracle's.
* EQR-SYEV: within 100 n u kappa(A) kappa(R) of the oracle's EQR-SYEV (the eigenvector error grows
  with kappa(A), Section 5); its residual is the one that is not constant (Section 7: proportional to
  kappa(A)^{1/2}, even for random matrices), so its bar is 100 u kappa(A)^{1/2}; at half the row count (m = 4096, the same spectrum and Z recipe,
  kappa(Z) = 1e4): the library's cyclic Jacobi eigensolver (a comparison baseline, one launch pair per
  rotation round) takes about 35 s per call at m = 4096 and more than three minutes at m = 8192,
  beyond a test's time.  The eigendecomposition does not depend on Z; everything after it (the
  Householder QR and the substitution) runs at the full size in the other variants.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from oracle import metrics, reference, variants

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")

M, N, KAPPA_A = 8192, 64, 1e6
KZ = [1e1, 1e4, 1e7]
_cache = {}


@pytest.fixture(scope="module")
def dense_a():
    banner("config2: generating A (m = 8192, Haar eigenvectors) on the host")
    a, _, _ = W.dense_spd(W.rng_for(2, 0, M, N), M, KAPPA_A, kind="haar")
    return a, to_dev(a)


def _z(kz):
    if ("z", kz) not in _cache:
        _cache[("z", kz)] = W.tall_skinny(W.rng_for(2, 1, M, N, int(np.log10(kz))), M, N, kz)
    return _cache[("z", kz)]


def _oracle(name, a, kz):
    key = (name, kz)
    if key not in _cache:
        z = _z(kz)
        if name == "chol_eqr":
            _cache[key] = reference.chol_eqr(a, z)
        elif name == "eqr_syev":
            _cache[key] = reference.eqr_syev(a, z)
        elif name == "cholqr":
            _cache[key] = variants.cholqr(a, z, gram="upper")
        else:
            _cache[key] = variants.VARIANTS[name](a, z)
    return _cache[key]


def _gpu(alg, A, z, **kw):
    q, r = getattr(oqr, alg)(A, to_dev_colmajor(z), **kw)
    return to_host(q), to_host(r)


def _common(a, z, q, r, res_bar=1e-12):
    assert metrics.residual_f(z, q, r) <= res_bar
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)


@pytest.mark.parametrize("pass1", ["fp64", "bf16x2", "bf16x3"])
@pytest.mark.parametrize("kz", KZ)
def test_config2_cholqr2(dense_a, kz, pass1):
    a, A = dense_a
    z = _z(kz)
    banner(f"config2 cholqr2 kz={kz:g} pass1={pass1}")
    q, r = _gpu("cholqr2", A, z, pass1=pass1, pass2="fp64")
    _, r0 = _oracle("chol_eqr", a, kz)
    kap = np.linalg.cond(r0)
    _common(a, z, q, r)
    loss = metrics.orth_loss(a, q)
    if pass1 != "fp64":
        from oracle import mixed
        banner(f"config2 cholqr2 kz={kz:g} pass1={pass1}: CPU emulation of the schedule")
        qe, _, info = mixed.cholqr2(a, z, pass1, "fp64", symmetric_blocks=64)
        assert info == 0
        assert loss <= max(1e-12, 10 * metrics.orth_loss(a, qe)), loss
        assert metrics.r_forward_error(r, r0) <= 10 * N * U * kap + kap * loss
    else:
        assert loss <= 1e-12
        assert metrics.r_forward_error(r, r0) <= 10 * N * U * kap


@pytest.mark.parametrize("kz", KZ)
def test_config2_cholqr_single_pass(dense_a, kz):
    a, A = dense_a
    z = _z(kz)
    banner(f"config2 cholqr kz={kz:g}")
    q, r = _gpu("cholqr", A, z)
    q0, r0 = _oracle("cholqr", a, kz)
    _common(a, z, q, r)
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + 1e-13
    kap = np.linalg.cond(r0)
    assert metrics.r_forward_error(r, r0) <= max(10 * N * U * kap, 10 * U * kap ** 2)


@pytest.mark.parametrize("kz", KZ)
def test_config2_pre_cholqr(dense_a, kz):
    a, A = dense_a
    z = _z(kz)
    banner(f"config2 pre_cholqr kz={kz:g}")
    q, r = _gpu("pre_cholqr", A, z)
    q0, r0 = _oracle("pre_cholqr", a, kz)
    _common(a, z, q, r)
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + 1e-13
    assert metrics.r_forward_error(r, r0) <= 100 * N * U * KAPPA_A * np.linalg.cond(r0)


@pytest.mark.parametrize("kz", KZ)
def test_config2_chol_a(dense_a, kz):
    a, A = dense_a
    z = _z(kz)
    banner(f"config2 chol_a kz={kz:g}")
    q, r = _gpu("chol_a", A, z)
    q0, r0 = _oracle("chol_eqr", a, kz)
    _common(a, z, q, r)
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + 1e-13
    tol = 100 * N * U * np.sqrt(KAPPA_A) * np.linalg.cond(r0)
    assert metrics.r_forward_error(r, r0) <= tol
    assert np.abs(q - q0).max() <= tol * np.abs(q0).max()


@pytest.mark.parametrize("variant", ["cgs", "mgs_row", "mgs_col", "cgs2"])
@pytest.mark.parametrize("kz", KZ)
def test_config2_gram_schmidt(dense_a, kz, variant):
    a, A = dense_a
    z = _z(kz)
    banner(f"config2 gs {variant} kz={kz:g}: CPU run of the same algorithm")
    q0, r0 = _oracle(variant, a, kz)
    banner(f"config2 gs {variant} kz={kz:g}: GPU")
    q, r = _gpu("gs", A, z, variant=variant)
    _common(a, z, q, r)
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + 1e-13
    kap = np.linalg.cond(r0)
    bound = 10 * U * kap ** 2 if variant == "cgs" else 100 * N * U * kap
    assert metrics.r_forward_error(r, r0) <= max(bound, 100 * N * U * kap)


def test_config2_eig_a_half_size():
    m = 4096
    banner("config2 eig_a m=4096: generating A (Haar eigenvectors)")
    a, _, _ = W.dense_spd(W.rng_for(2, 0, m, N), m, KAPPA_A, kind="haar")
    z = W.tall_skinny(W.rng_for(2, 1, m, N, 4), m, N, 1e4)
    banner("config2 eig_a m=4096 kz=1e4: GPU (cyclic Jacobi)")
    q, r = _gpu("eig_a", to_dev(a), z)
    banner("config2 eig_a m=4096 kz=1e4: CPU run of the same algorithm")
    q0, r0 = reference.eqr_syev(a, z)
    _common(a, z, q, r, res_bar=max(1e-12, 100 * U * np.sqrt(KAPPA_A)))
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + 1e-13
    tol = 100 * N * U * KAPPA_A * np.linalg.cond(r0)
    assert metrics.r_forward_error(r, r0) <= tol
    assert np.abs(q - q0).max() <= tol * np.abs(q0).max()
