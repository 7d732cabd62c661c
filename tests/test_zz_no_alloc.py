"""The allocation-free CholQR2-A entry point (oqr_cholqr2_noalloc) against oqr_cholqr2.

Both run the same kernels in the same order, one on the caller's workspace and
one on the library's fixed device scratch, so Q, R and info must agree bit for
bit; each result is also held to the CholQR2-A tolerances against the oracle
(residual and A-orthogonality <= 1e-12, R forward error <= 10 n u kappa).
Consecutive calls reuse the scratch with its previous contents: the second call
of each sequence is smaller than the first.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from oracle import metrics, reference

pytestmark = pytest.mark.gpu

oqr = pytest.importorskip("paper_1401_5171_amd")


def _empty_like_cols(m, n):
    import torch
    return torch.empty(n, m, dtype=torch.float64, device="cuda").t()


def _call_noalloc(A, Z, n, **kw):
    import torch
    m = Z.shape[0]
    Q, R = _empty_like_cols(m, n), _empty_like_cols(n, n)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    oqr.cholqr2_noalloc_into(A, Z, Q, R, info, **kw)
    torch.cuda.synchronize()
    return to_host(Q), to_host(R), int(info.item())


def _call_ws(A, Z, n, **kw):
    import torch
    m = Z.shape[0]
    plan = oqr.Plan("cholqr2", A, n, **kw)
    Q, R = _empty_like_cols(m, n), _empty_like_cols(n, n)
    plan.run(Z, Q, R)
    torch.cuda.synchronize()
    return to_host(Q), to_host(R), int(plan.info.item())


def _dense(cfg, m, n, ka, kz):
    rng = W.rng_for(cfg, 0, m, n)
    a, _, _ = W.dense_spd(rng, m, ka)
    z = W.tall_skinny(rng, m, n, kz)
    return a, z


def _check_against_oracle(z, q, r, r0):
    n = z.shape[1]
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0) + 1e-15
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)


@pytest.mark.parametrize("pass1", ["fp64", "bf16x2"])
def test_noalloc_matches_workspace_entry_dense(pass1):
    """Two calls in a row on the same device scratch, the second smaller (2048 x 64, then 700 x 20)."""
    for (m, n) in [(2048, 64), (700, 20)]:
        a, z = _dense(93, m, n, 1e6, 1e4)
        A, Z = to_dev(a), to_dev_colmajor(z)
        banner(f"noalloc dense m={m} n={n} pass1={pass1}")
        qn, rn, infon = _call_noalloc(A, Z, n, pass1=pass1)
        qw, rw, infow = _call_ws(A, Z, n, pass1=pass1)
        assert infon == 0 and infow == 0
        assert np.array_equal(qn, qw) and np.array_equal(rn, rw)
        _, r0 = reference.chol_eqr(a, z)
        _check_against_oracle(z, qn, rn, r0)
        assert metrics.orth_loss(a, qn) <= 1e-12


def test_noalloc_matches_workspace_entry_stencil_then_smaller_dense():
    """A stencil operator (fused Gram path), then a smaller dense problem on the same scratch."""
    nx, ny, nz, n = 20, 16, 12, 32
    m = nx * ny * nz
    rng = W.rng_for(94, 0, m, n)
    z = W.tall_skinny(rng, m, n, 1e3)
    st = W.laplacian7(nx, ny, nz)
    op = oqr.Stencil7(nx, ny, nz, st.center, st.off)
    Z = to_dev_colmajor(z)
    banner(f"noalloc stencil {nx}x{ny}x{nz} n={n}")
    qn, rn, infon = _call_noalloc(op, Z, n)
    qw, rw, infow = _call_ws(op, Z, n)
    assert infon == 0 and infow == 0
    assert np.array_equal(qn, qw) and np.array_equal(rn, rw)
    q0, r0 = reference.stencil_eqr(st, z)
    _check_against_oracle(z, qn, rn, r0)
    assert metrics.orth_loss(st, qn) <= 1e-12

    a, z2 = _dense(95, 300, 9, 1e4, 1e3)
    A, Z2 = to_dev(a), to_dev_colmajor(z2)
    banner("noalloc dense m=300 n=9 after the stencil")
    qn, rn, infon = _call_noalloc(A, Z2, 9)
    qw, rw, infow = _call_ws(A, Z2, 9)
    assert infon == 0 and infow == 0
    assert np.array_equal(qn, qw) and np.array_equal(rn, rw)
    _, r0 = reference.chol_eqr(a, z2)
    _check_against_oracle(z2, qn, rn, r0)
    assert metrics.orth_loss(a, qn) <= 1e-12


def test_noalloc_in_place_and_oversize_rejected():
    import torch
    a, z = _dense(96, 1000, 40, 1e5, 1e3)
    A, Z = to_dev(a), to_dev_colmajor(z)
    R = _empty_like_cols(40, 40)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    banner("noalloc in place")
    oqr.cholqr2_noalloc_into(A, Z, Z, R, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    q, r = to_host(Z), to_host(R)
    assert metrics.residual_f(z, q, r) <= 1e-12 and metrics.orth_loss(a, q) <= 1e-12

    # a request whose workspace exceeds the fixed scratch is refused before anything is enqueued
    nx, ny, nz, n = 128, 128, 16, 64
    m = nx * ny * nz
    op, _ = oqr.make_op(oqr.Stencil7(nx, ny, nz, 6.001, -1.0))
    need = oqr.lib().oqr_workspace_bytes(oqr.ALG["cholqr2"], ctypes.byref(op), m, n, None)
    assert need > oqr.noalloc_scratch_bytes()
    Zb = torch.zeros(n, m, dtype=torch.float64, device="cuda").t()
    Qb = torch.zeros(n, m, dtype=torch.float64, device="cuda").t()
    Rb = torch.zeros(n, n, dtype=torch.float64, device="cuda").t()
    info.fill_(-7)
    banner("noalloc oversize request")
    with pytest.raises(oqr.OQRError) as e:
        oqr.cholqr2_noalloc_into(oqr.Stencil7(nx, ny, nz, 6.001, -1.0), Zb, Qb, Rb, info)
    assert e.value.status == oqr.OQR_E_SCRATCH
    torch.cuda.synchronize()
    assert int(info.item()) == -7          # nothing was enqueued
