"""GPU parity of PRE-CHOLQR-A (Algorithm 2, Section 3): Householder QR of Z in the Euclidean product,
CHOLQR-A on the orthonormal factor, R = S U.

Bars: residual <= 1e-12; orthogonality within 10x (plus a floor) of the oracle's run of the same
algorithm, and below the Section 3 level c u kappa(A) when kappa(Z) is far beyond what CHOLQR-A
survives; R against the oracle within n u kappa(A) kappa(R) (the CHOLQR-A step sees
kappa(A^{1/2} Y) <= kappa(A)^{1/2}).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from oracle import metrics, reference, variants

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")


def case(cfg, m, n, ka, kz, seed=0):
    rng = W.rng_for(cfg, seed, m, n)
    a, _, _ = W.dense_spd(rng, m, ka)
    z = W.tall_skinny(rng, m, n, kz)
    return a, z


def check_against_oracle(a, z, q, r):
    q0, r0 = variants.pre_cholqr(a, z)
    n = z.shape[1]
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert metrics.orth_loss(a, q) <= 10 * metrics.orth_loss(a, q0) + 1e-13
    ka = np.linalg.cond(a) if not hasattr(a, "nx") else 1e4
    assert metrics.r_forward_error(r, r0) <= 100 * n * U * ka * np.linalg.cond(r0)


def test_pre_cholqr_config1():
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    banner("pre_cholqr config1")
    q, r = (to_host(x) for x in oqr.pre_cholqr(to_dev(a), to_dev_colmajor(z)))
    check_against_oracle(a, z, q, r)
    # the stable class at this size (Section 3): orthogonality at the FP64 level
    assert metrics.orth_loss(a, q) <= 1e-12


def test_identity_operator_is_householder_qr():
    """A = I: PRE-CHOLQR reduces to the Euclidean Householder QR (sign-fixed numpy.linalg.qr)."""
    m, n = 300, 17
    z = W.tall_skinny(W.rng_for(70), m, n, 1e6)
    banner("pre_cholqr A = I")
    q, r = (to_host(x) for x in oqr.pre_cholqr(to_dev(np.eye(m)), to_dev_colmajor(z)))
    qn, rn = np.linalg.qr(z)
    sg = np.sign(np.diag(rn))
    qn, rn = qn * sg, (rn.T * sg).T
    assert metrics.r_forward_error(r, rn) <= 100 * n * U * np.linalg.cond(rn)
    assert np.abs(q - qn).max() <= 100 * n * U * np.linalg.cond(rn)
    assert np.linalg.norm(q.T @ q - np.eye(n)) <= 1e-13


def test_survives_where_cholqr_breaks_down():
    """kappa(Z) = 1e12, kappa(A) = 1e2: CHOLQR-A's Gram is numerically singular (its Cholesky fails
    or loses all orthogonality), PRE-CHOLQR keeps the loss at c u kappa(A)."""
    a, z = case(71, 800, 24, 1e2, 1e12)
    banner("pre_cholqr kappa(Z) = 1e12")
    q, r = (to_host(x) for x in oqr.pre_cholqr(to_dev(a), to_dev_colmajor(z)))
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(a, q) <= 1e-12
    q1, r1, info = variants.cholqr(a, z, return_info=True)
    assert info > 0 or metrics.orth_loss(a, q1) > 1e-3


@pytest.mark.parametrize("m,n", [(1, 1), (65, 64), (1531, 129), (2048, 256)])
def test_pre_cholqr_ragged(m, n):
    a, z = case(72, m, n, 1e3, 1e4 if n > 1 else 1.0)
    banner(f"pre_cholqr m={m} n={n}")
    q, r = (to_host(x) for x in oqr.pre_cholqr(to_dev(a), to_dev_colmajor(z)))
    check_against_oracle(a, z, q, r)


def test_pre_cholqr_stencil():
    st = W.laplacian7(12, 10, 9)
    z = W.tall_skinny(W.rng_for(73), st.m, 30, 1e8)
    banner("pre_cholqr stencil")
    q, r = (to_host(x) for x in oqr.pre_cholqr(oqr.Stencil7(12, 10, 9, st.center, st.off), to_dev_colmajor(z)))
    q0, r0 = variants.pre_cholqr(st, z)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= 10 * metrics.orth_loss(st, q0) + 1e-13
    assert metrics.r_forward_error(r, r0) <= 100 * 30 * U * 1e3 * np.linalg.cond(r0)


def test_pre_cholqr_in_place():
    a, z = case(74, 400, 12, 1e3, 1e5)
    Z = to_dev_colmajor(z)
    plan = oqr.Plan("pre_cholqr", to_dev(a), 12)
    import torch
    R = torch.empty(12, 12, dtype=torch.float64, device="cuda").t()
    plan.run(Z, Z, R)
    torch.cuda.synchronize()
    assert int(plan.info.item()) == 0
    check_against_oracle(a, z, to_host(Z), to_host(R))


def identity_op(m):
    """A = I as a tridiagonal operator (d = 1, e = 0): PRE-CHOLQR is then the Euclidean QR itself."""
    return oqr.Tridiag(np.ones(m), np.zeros(m - 1))


def lapack_qr(z):
    qn, rn = np.linalg.qr(z)
    sg = np.where(np.diag(rn) < 0, -1.0, 1.0)
    return qn * sg, (rn.T * sg).T


@pytest.mark.parametrize("m,n", [(1029, 64), (100000, 64), (70001, 16), (5000, 33), (3000, 1), (20000, 40),
                                 (300, 64), (257, 64)])
def test_euclidean_qr_tree_against_lapack(m, n):
    """The Euclidean QR for n <= 64 is a tree of Householder QRs (blocks of 256-1024 rows, their
    triangles stacked level by level): against LAPACK's QR of the same Z, sign-fixed, with one or
    several levels, a last block with fewer rows than n (1029 = 4 * 256 + 5; 257), a single block
    (300) and n = 1."""
    z = W.tall_skinny(W.rng_for(75, m, n), m, n, 1e6 if n > 1 else 1.0)
    qn, rn = lapack_qr(z)
    banner(f"euclidean qr tree m={m} n={n}")
    q, r = (to_host(x) for x in oqr.pre_cholqr(identity_op(m), to_dev_colmajor(z)))
    bar = 100 * n * U * np.linalg.cond(rn)
    assert metrics.r_forward_error(r, rn) <= bar
    assert np.abs(q - qn).max() <= bar
    assert np.linalg.norm(q.T @ q - np.eye(n)) <= 1e-13 * max(1, n / 8)
    assert metrics.residual_f(z, q, r) <= 1e-13


@pytest.mark.parametrize("m,n", [(3000, 8), (40000, 48)])
def test_euclidean_qr_rank_deficient(m, n):
    """A zero column and a repeated column: the Householder factor stays orthonormal (tau = 0 for the
    zero column, as in LAPACK), Z = Q R holds, and the Cholesky step of PRE-CHOLQR sees Y^T Y = I."""
    z = W.tall_skinny(W.rng_for(76, m, n), m, n, 1e2)
    z[:, 3] = 0.0
    z[:, 5] = z[:, 1]
    banner(f"euclidean qr rank deficient m={m} n={n}")
    Q, R = oqr.pre_cholqr(identity_op(m), to_dev_colmajor(z))
    q, r = to_host(Q), to_host(R)
    assert np.all(np.isfinite(q)) and np.all(np.isfinite(r))
    assert np.linalg.norm(q.T @ q - np.eye(n)) <= 1e-13
    assert metrics.residual_f(z, q, r) <= 1e-13
    assert abs(r[3, 3]) <= 1e-13 * np.abs(r).max() and abs(r[5, 5]) <= 1e-13 * np.abs(r).max()
