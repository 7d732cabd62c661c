"""GPU generalised least squares (Section 1): x = R^{-1} Q^T A b minimises ||Z x - b||_A.

The factorisation comes from the GPU (CholQR2-A); the oracle's answer is computed independently by
whitening (A = C^T C, LAPACK least squares on C Z, C b).  Bars: against the same formula evaluated on
the CPU from the GPU's own Q and R, n u kappa(R) (this step's arithmetic); against the whitening
solution, the least-squares perturbation bound u (kappa + kappa^2 rho) with kappa = kappa(R) and
rho = ||C (Z x - b)|| / (||C Z|| ||x||), times 100 n.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from oracle import reference, stencil

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")
torch = pytest.importorskip("torch")


def ls_bound(a_dense, z, x, b, kr, n):
    c = np.linalg.cholesky(a_dense).T
    r = c @ (z @ x - b)
    rho = np.linalg.norm(r) / (np.linalg.norm(c @ z, 2) * max(np.linalg.norm(x), 1e-300))
    return 100 * n * U * (kr + kr * kr * rho)


def test_gls_dense_several_right_hand_sides():
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    b = np.random.default_rng(21).standard_normal((500, 3))
    A = to_dev(a)
    banner("gls dense")
    Q, R = oqr.cholqr2(A, to_dev_colmajor(z))
    x = to_host(oqr.gls(A, Q, R, to_dev_colmajor(b)))
    q, r = to_host(Q), to_host(R)
    kr = np.linalg.cond(r)
    xf = np.linalg.solve(r, q.T @ (a @ b))                # the formula, on the CPU, same Q and R
    assert np.abs(x - xf).max() <= 10 * 20 * U * kr * np.abs(xf).max()
    x0 = reference.gls(a, z, b)
    for j in range(3):
        assert np.abs(x[:, j] - x0[:, j]).max() <= ls_bound(a, z, x0[:, j], b[:, j], kr, 20) * np.abs(x0[:, j]).max()


def test_gls_exact_range_and_vector_input():
    rng = W.rng_for(22)
    a, _, _ = W.dense_spd(rng, 300, 1e3)
    z = W.tall_skinny(rng, 300, 8, 1e2)
    xs = np.linspace(-1.0, 2.0, 8)
    A = to_dev(a)
    Q, R = oqr.cholqr2(A, to_dev_colmajor(z))
    b = torch.from_numpy(z @ xs).cuda()
    x = to_host(oqr.gls(A, Q, R, b))
    assert x.shape == (8,)
    assert np.abs(x - xs).max() <= 100 * 8 * U * np.linalg.cond(to_host(R)) * np.abs(xs).max()


def test_gls_stencil():
    st = W.laplacian7(10, 9, 8)
    rng = W.rng_for(23)
    z = W.tall_skinny(rng, st.m, 12, 1e2)
    b = np.random.default_rng(24).standard_normal((st.m, 2))
    op = oqr.Stencil7(10, 9, 8, st.center, st.off)
    banner("gls stencil")
    Q, R = oqr.cholqr2(op, to_dev_colmajor(z))
    x = to_host(oqr.gls(op, Q, R, to_dev_colmajor(b)))
    x0 = reference.gls(st, z, b)
    kr = np.linalg.cond(to_host(R))
    ad = stencil.dense(st)
    for j in range(2):
        assert np.abs(x[:, j] - x0[:, j]).max() <= ls_bound(ad, z, x0[:, j], b[:, j], kr, 12) * np.abs(x0[:, j]).max()


def test_gls_argument_errors():
    a = to_dev(np.eye(16))
    Q = torch.zeros(8, 16, dtype=torch.float64, device="cuda").t()
    R = torch.eye(8, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        oqr.gls(a, Q, R, torch.zeros(15, dtype=torch.float64, device="cuda"))
