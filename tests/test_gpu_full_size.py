"""Parity at the full sizes of the timed workloads, built and launched exactly as bench.py does.

The oracle cannot factor these sizes in a test's time, so the checks are properties that fix the
result at any size, evaluated on the CPU from the device's Q and R with the oracle's metrics:
the residual ||Z - QR||_F / ||Z||_F, the A-orthogonality ||I - Q^T A Q||_2, R upper triangular with
a positive diagonal, and the schedules' R against each other (R is unique, Section 2): mixed with
a hi/lo (bf16x2, the bench's) or three-slice first pass, and FP64. The
batch is checked instance by instance on a spread sample, each against the oracle's CHOL-EQR.
Inputs come from the seeded generators only (no method arithmetic); A of the dense workload and
the batch instances are formed on the device by the generators' torch path, as in the bench.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_host
from oracle import metrics, reference

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")
torch = pytest.importorskip("torch")


def _schedules(A, Z, n):
    out = {}
    for name, p1 in (("mixed", "bf16x2"), ("mixed3", "bf16x3"), ("fp64", "fp64")):
        plan = oqr.Plan("cholqr2", A, n, pass1=p1, pass2="fp64")
        q, r = plan(Z)
        torch.cuda.synchronize()
        out[name] = (to_host(q), to_host(r))
    return out


def _check_r(r):
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)


def test_dense_m32768_n256_full_size():
    """Dense SPD A (m = 32768, kappa 1e8, butterfly eigenvectors), Z with kappa 1e5, n = 256."""
    m, n = 32768, 256
    dev = torch.device("cuda", 0)
    rng = W.rng_for(4, 0)
    banner("full size dense m=32768 n=256: generating A on the device")
    A, _, _ = W.dense_spd_device(rng, m, 1e8, dev)
    z = W.tall_skinny(rng, m, n, 1e5)
    Z = torch.from_numpy(np.ascontiguousarray(z.T)).to(dev).t()
    banner("full size dense: CholQR2 mixed and FP64")
    res = _schedules(A, Z, n)
    a = to_host(A)
    del A
    torch.cuda.empty_cache()
    for name, (q, r) in res.items():
        banner(f"full size dense: CPU checks ({name})")
        _check_r(r)
        assert metrics.residual_f(z, q, r) <= 1e-12, name
        assert metrics.orth_loss(a, q) <= 1e-12, name
    r64 = res["fp64"][1]
    for name in ("mixed", "mixed3"):
        assert metrics.r_forward_error(res[name][1], r64) <= 20 * n * U * np.linalg.cond(r64), name


def test_stencil_128x128x64_n128_full_size():
    """7-point Laplacian + 1e-3 I on 128 x 128 x 64 (m = 2^20), n = 128, column-scaled Z (kappa 1e4)."""
    nx, ny, nz, n = 128, 128, 64, 128
    st = W.laplacian7(nx, ny, nz)
    z = W.gaussian_scaled(W.rng_for(3, 0), st.m, n, 1e4)
    Z = torch.from_numpy(np.ascontiguousarray(z.T)).cuda().t()
    banner("full size stencil 128x128x64 n=128: CholQR2 mixed and FP64")
    res = _schedules(oqr.Stencil7(nx, ny, nz, st.center, st.off), Z, n)
    for name, (q, r) in res.items():
        banner(f"full size stencil: CPU checks ({name})")
        _check_r(r)
        assert metrics.residual_f(z, q, r) <= 1e-12, name
        assert metrics.orth_loss(st, q) <= 1e-12, name
    r64 = res["fp64"][1]
    for name in ("mixed", "mixed3"):
        assert metrics.r_forward_error(res[name][1], r64) <= 20 * n * U * np.linalg.cond(r64), name


def test_stencil_3b_haar_mixed_full_grid():
    """The stress variant of the stencil workload on the full 128 x 128 x 64 grid: Z = U diag(s) W^T
    with Haar U, W and kappa(Z) = 1e4 (column scaling no longer hides the conditioning).  CholQR2-A
    (bf16x2, bf16x3 and FP64 first pass) against the exact-eigenbasis EQR-SYEV oracle; one FP64 CHOLQR
    pass against the same algorithm on the CPU (its loss grows like kappa(A^{1/2} Z)^2 u)."""
    from oracle import variants
    nx, ny, nz, n = 128, 128, 64, 128
    st = W.laplacian7(nx, ny, nz)
    banner("full grid 3b: generating Haar-mixed Z")
    z = W.tall_skinny(W.rng_for(3, 7), st.m, n, 1e4)
    Z = torch.from_numpy(np.ascontiguousarray(z.T)).cuda().t()
    op = oqr.Stencil7(nx, ny, nz, st.center, st.off)
    banner("full grid 3b: CholQR2 mixed and FP64")
    res = _schedules(op, Z, n)
    banner("full grid 3b: single FP64 pass")
    q1, r1 = (to_host(x) for x in oqr.cholqr(op, Z))
    del Z
    torch.cuda.empty_cache()
    banner("full grid 3b: oracle (exact-eigenbasis EQR-SYEV)")
    _, r0 = reference.stencil_eqr(st, z)
    kap = np.linalg.cond(r0)
    for name, (q, r) in res.items():
        banner(f"full grid 3b: CPU checks ({name})")
        _check_r(r)
        assert metrics.residual_f(z, q, r) <= 1e-12, name
        assert metrics.orth_loss(st, q) <= 1e-12, name
        assert metrics.r_forward_error(r, r0) <= 10 * n * U * kap, name
    del res
    banner("full grid 3b: CPU run of CHOLQR-A")
    qc, _ = variants.cholqr(st, z, gram="upper")
    _check_r(r1)
    assert metrics.residual_f(z, q1, r1) <= 1e-12
    assert metrics.orth_loss(st, q1) <= 10 * metrics.orth_loss(st, qc) + 1e-13


def _batch_full_size(dtype):
    dev = torch.device("cuda", 0)
    sizes = W.batch_plan(4096)
    banner(f"full size batch {dtype}: generating 4096 instances on the device")
    As, Zs = [], []
    for k, p in enumerate(sizes):
        a, zz = W.batch_instance_device(p, dev, dtype)
        As.append(a)
        Zs.append(zz)
        if (k + 1) % 1024 == 0:
            banner(f"full size batch: generated {k + 1}")
    plan = oqr.BatchPlan(As, Zs)
    banner("full size batch: one launch")
    plan.run()
    torch.cuda.synchronize()
    return plan, As, Zs


def test_batch_4096_full_size_sampled():
    """The 4096-instance batch (m log-uniform in [256, 4096], n in {8, 16, 32, 64}, kappa(A) in
    [1e2, 1e8]) in one launch; every info word zero, and 13 instances spread over the batch checked
    one by one against CHOL-EQR."""
    plan, As, Zs = _batch_full_size(torch.float64)
    info = to_host(plan.info)
    assert np.all(info == 0), np.nonzero(info)
    for k in range(0, 4096, 320):
        a, z = to_host(As[k]), to_host(Zs[k])
        q, r = to_host(plan.Qs[k]), to_host(plan.Rs[k])
        n = z.shape[1]
        banner(f"full size batch: instance {k} (m={a.shape[0]}, n={n}) against the oracle")
        q0, r0 = reference.chol_eqr(a, z)
        aq2 = metrics.diagnostics(a, z, q0, r0)["a_q2"]
        _check_r(r)
        assert metrics.residual_f(z, q, r) <= 1e-12, k
        assert metrics.orth_loss(a, q) <= max(1e-12, 100 * U * aq2 * n), k
        assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0) + 1e-15, k
    del plan, As, Zs
    torch.cuda.empty_cache()


def test_batch_4096_full_size_fp32_storage_sampled():
    """The same batch with FP32 storage (A_i, Z_i rounded to FP32; the kernel widens to FP64 and rounds
    Q_i, R_i to FP32 on store).  The oracle factors the rounded inputs widened to FP64, so the input
    rounding is not charged: orthogonality <= max(1e-6, 10 u32 ||A|| ||Q||^2), residual <= 1e-6 (Q and
    R are stored in FP32), R within the FP32 storage error of the oracle's; 13 instances sampled."""
    u32 = 2.0 ** -24
    plan, As, Zs = _batch_full_size(torch.float32)
    info = to_host(plan.info)
    assert np.all(info == 0), np.nonzero(info)
    for k in range(0, 4096, 320):
        a32 = to_host(As[k]).astype(np.float64)
        z32 = to_host(Zs[k]).astype(np.float64)
        q = to_host(plan.Qs[k]).astype(np.float64)
        r = to_host(plan.Rs[k]).astype(np.float64)
        n = z32.shape[1]
        banner(f"full size batch fp32: instance {k} (m={a32.shape[0]}, n={n}) against the oracle")
        q0, r0 = reference.chol_eqr(a32, z32)
        aq2 = metrics.diagnostics(a32, z32, q0, r0)["a_q2"]
        _check_r(r)
        assert metrics.orth_loss(a32, q) <= max(1e-6, 10 * u32 * aq2), k
        assert metrics.residual_f(z32, q, r) <= 1e-6, k
        assert metrics.r_forward_error(r, r0) <= 1e-5 * max(1.0, np.linalg.cond(r0) * u32 * 1e3), k
    del plan, As, Zs
    torch.cuda.empty_cache()
