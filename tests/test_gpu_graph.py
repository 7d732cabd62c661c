"""CholQR2-A captured in a HIP graph (`Plan.capture`): every replay equals the eager call bit for bit.

The graph is replayed several times with eager work (Q cleared) and synchronisations between the
replays; then Z is overwritten with a new matrix and the replay must equal an eager call on that
matrix, and match the oracle's CHOL-EQR within the FP64 tolerances.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_host
from oracle import metrics, reference

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")
torch = pytest.importorskip("torch")


def _colmajor(z):
    return torch.from_numpy(np.ascontiguousarray(z.T)).cuda().t()


def _replays_match(plan, Z, m, n, znew, oracle_qr):
    Q = torch.empty(n, m, dtype=torch.float64, device="cuda").t()
    R = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
    plan.run(Z, Q, R)
    torch.cuda.synchronize()
    q0, r0 = Q.clone(), R.clone()
    g = plan.capture(Z, Q, R)
    for rep in range(3):
        Q.zero_()
        R.zero_()
        plan.info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(plan.info.item()) == 0, rep
        assert torch.equal(Q, q0) and torch.equal(R, r0), rep
    # new data in the captured input
    Z.copy_(_colmajor(znew))
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    q1, r1 = Q.clone(), R.clone()
    Q2 = torch.empty(n, m, dtype=torch.float64, device="cuda").t()
    R2 = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
    plan.run(Z, Q2, R2)
    torch.cuda.synchronize()
    assert torch.equal(q1, Q2) and torch.equal(r1, R2)
    qh, rh = to_host(q1), to_host(r1)
    qo, ro = oracle_qr(znew)
    assert metrics.residual_f(znew, qh, rh) <= 1e-12
    assert metrics.r_forward_error(rh, ro) <= 10 * n * U * np.linalg.cond(ro)
    return qh


def test_dense_cholqr2_mixed_graph_replays():
    m, n = 700, 24
    rng = W.rng_for(1, 40, m, n)
    a, _, _ = W.dense_spd(rng, m, 1e4)
    z = W.tall_skinny(rng, m, n, 1e3)
    znew = W.tall_skinny(rng, m, n, 1e3)
    A = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    plan = oqr.Plan("cholqr2", A, n, pass1="bf16x2", pass2="fp64")
    banner("graph: dense cholqr2 bf16x2 + fp64, m=700 n=24")
    q = _replays_match(plan, _colmajor(z), m, n, znew, lambda zz: reference.chol_eqr(a, zz))
    assert metrics.orth_loss(a, q) <= 1e-12


def test_stencil_cholqr2_graph_replays():
    grid, n = (20, 16, 12), 40
    st = W.laplacian7(*grid)
    rng = W.rng_for(3, 41, n)
    z = W.tall_skinny(rng, st.m, n, 1e3)
    znew = W.tall_skinny(rng, st.m, n, 1e3)
    plan = oqr.Plan("cholqr2", oqr.Stencil7(*grid, st.center, st.off), n)
    banner("graph: stencil cholqr2 fp64, 20x16x12 n=40")
    q = _replays_match(plan, _colmajor(z), st.m, n, znew, lambda zz: reference.stencil_eqr(st, zz))
    assert metrics.orth_loss(st, q) <= 1e-12
