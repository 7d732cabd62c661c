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


def test_batch_4096_full_size_sampled():
    """The 4096-instance batch (m log-uniform in [256, 4096], n in {8, 16, 32, 64}, kappa(A) in
    [1e2, 1e8]) in one launch; every info word zero, and 13 instances spread over the batch checked
    one by one against CHOL-EQR."""
    dev = torch.device("cuda", 0)
    sizes = W.batch_plan(4096)
    banner("full size batch: generating 4096 instances on the device")
    As, Zs = [], []
    for k, p in enumerate(sizes):
        a, zz = W.batch_instance_device(p, dev, torch.float64)
        As.append(a)
        Zs.append(zz)
        if (k + 1) % 1024 == 0:
            banner(f"full size batch: generated {k + 1}")
    plan = oqr.BatchPlan(As, Zs)
    banner("full size batch: one launch")
    plan.run()
    torch.cuda.synchronize()
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
