"""GPU parity of the batched CholQR2-A (one persistent launch) against the CPU oracle.

Instances follow the batch workload's recipe (log-uniform m, n in {8, 16, 32, 64}, kappa(A)
log-uniform, Gaussian Z, butterfly eigenvectors) at sizes the oracle finishes in seconds, plus
ragged n.  FP64 storage: residual and orthogonality <= 1e-12 where u ||A|| ||Q||^2 allows it
(the stable class), R forward error <= 10 n u kappa(R) against CHOL-EQR.  FP32 storage: the oracle
runs on the FP32-rounded inputs widened to FP64; orthogonality <= max(1e-6, 10 u32 ||A|| ||Q||^2).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_host
from oracle import metrics, reference, variants

pytestmark = pytest.mark.gpu
oqr = pytest.importorskip("paper_1401_5171_amd")
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


def make_batch(count, m_lo=32, m_hi=600, n_set=(8, 16, 32, 64), k=(1e2, 1e6), extra_n=(), seed=7):
    plan = W.batch_plan(count, m_lo, m_hi, n_set, k[0], k[1], cfg=50 + seed)
    insts = []
    for i, p in enumerate(plan):
        n = p.n if i >= len(extra_n) else extra_n[i]
        p = W.BatchInstance(p.index, max(p.m, n), n, p.kappa)
        a, z = W.batch_instance(p, cfg=50 + seed)
        insts.append((a, z))
    return insts


def upload(insts, dtype):
    As = [torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).cuda() for a, _ in insts]
    Zs = [torch.from_numpy(np.ascontiguousarray(z.astype(dtype).T)).cuda().t() for _, z in insts]
    return As, Zs


def check_fp64(insts, plan):
    info = to_host(plan.info)
    assert np.all(info == 0), info
    for k, (a, z) in enumerate(insts):
        q, r = to_host(plan.Qs[k]), to_host(plan.Rs[k])
        q0, r0 = reference.chol_eqr(a, z)
        aq2 = metrics.diagnostics(a, z, q0, r0)["a_q2"]
        n = z.shape[1]
        assert metrics.residual_f(z, q, r) <= 1e-12, k
        assert metrics.orth_loss(a, q) <= max(1e-12, 100 * U * aq2 * n), k
        assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0) + 1e-15, k
        assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0), k


def test_batch_fp64_matches_oracle():
    insts = make_batch(48, extra_n=(1, 3, 17, 33, 63, 64))
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs)
    banner("batch fp64 48 instances")
    plan.run()
    torch.cuda.synchronize()
    check_fp64(insts, plan)


def _tuning(shape=None, wg=None, sort=None):
    t = oqr.default_batch_tuning()
    d = t.to_dict()
    if shape is not None:
        d["shape"] = [[shape] * oqr.BATCH_NCLASSES for _ in range(oqr.BATCH_MBUCKETS)]
    if wg is not None:
        d["wg_per_cu"] = wg
    if sort is not None:
        d["sort"] = sort
    return oqr.BatchTuning.from_dict(d)


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_batch_every_tile_shape_matches_oracle(shape):
    """Each Gram-phase tile shape (128 x 32, 64 x 32, 128 x 16, 64 x 16 rows x K step) on every
    instance: results against CHOL-EQR, and two runs bit for bit equal (fixed order of the sums)."""
    insts = make_batch(24, seed=8, extra_n=(1, 7, 33))
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs, tuning=_tuning(shape=shape))
    banner(f"batch tile shape {oqr.BATCH_SHAPE_NAMES[shape]}")
    plan.run()
    torch.cuda.synchronize()
    check_fp64(insts, plan)
    q1 = [q.clone() for q in plan.Qs]
    plan.run()
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(plan.Qs[k], q1[k])


@pytest.mark.parametrize("wg,sort", [(1, 1), (3, 1), (2, 0)])
def test_batch_launch_configuration_keeps_the_bits(wg, sort):
    """Workgroups per compute unit and the order instances are taken in do not change any sum."""
    insts = make_batch(24, seed=8)
    As, Zs = upload(insts, np.float64)
    ref = oqr.BatchPlan(As, Zs, tuning=_tuning(shape=1))
    ref.run()
    plan = oqr.BatchPlan(As, Zs, tuning=_tuning(shape=1, wg=wg, sort=sort))
    banner(f"batch wg_per_cu={wg} sort={sort}")
    plan.run()
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(plan.Qs[k], ref.Qs[k]) and torch.equal(plan.Rs[k], ref.Rs[k])


def _split_tuning(split_m, parts, shape=None, wg=None):
    d = _tuning(shape=shape, wg=wg).to_dict()
    d["split_m"], d["parts"] = split_m, parts
    return oqr.BatchTuning.from_dict(d)


@pytest.mark.parametrize("parts", [1, 2, 3, 8])
def test_batch_split_instances_match_oracle(parts):
    """Cooperative instances: those with m >= 700 run each pass as `parts` Gram parts over interleaved
    row blocks (partial Grams summed in part order) taken by any workgroup of the persistent launch;
    every instance matches CHOL-EQR, ragged n included; two runs, and a run with one workgroup per
    compute unit (other workgroups take the parts), repeat the bits."""
    insts = make_batch(20, m_lo=100, m_hi=1500, seed=15, extra_n=(64, 1, 33, 17))
    assert sum(z.shape[0] >= 700 for _, z in insts) >= 4
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs, tuning=_split_tuning(700, parts))
    banner(f"batch split m>=700 parts={parts}")
    plan.run()
    torch.cuda.synchronize()
    check_fp64(insts, plan)
    q1 = [q.clone() for q in plan.Qs]
    r1 = [r.clone() for r in plan.Rs]
    plan.run()
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(plan.Qs[k], q1[k])
    one = oqr.BatchPlan(As, Zs, tuning=_split_tuning(700, parts, wg=1))
    one.run()
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(one.Qs[k], q1[k]) and torch.equal(one.Rs[k], r1[k]), k


def test_batch_split_most_instances():
    """Nearly every instance split (8 parts each): many pass-2 parts published while others are still
    in pass 1; results against the oracle."""
    insts = make_batch(40, m_lo=300, m_hi=900, seed=19, extra_n=(64, 40))
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs, tuning=_split_tuning(300, 8))
    banner("batch split 40 instances x 8 parts")
    plan.run()
    torch.cuda.synchronize()
    check_fp64(insts, plan)


def test_batch_split_fp32_storage_and_shapes():
    """The split path with FP32 storage and a non-default tile shape, against the oracle on the rounded
    inputs."""
    insts = make_batch(16, m_lo=100, m_hi=1200, seed=16, k=(1e2, 1e4))
    As, Zs = upload(insts, np.float32)
    plan = oqr.BatchPlan(As, Zs, tuning=_split_tuning(600, 4, shape=3))
    banner("batch split fp32")
    plan.run()
    torch.cuda.synchronize()
    assert np.all(to_host(plan.info) == 0)
    for k, (a, z) in enumerate(insts):
        a32 = a.astype(np.float32).astype(np.float64)
        z32 = z.astype(np.float32).astype(np.float64)
        q, r = to_host(plan.Qs[k]).astype(np.float64), to_host(plan.Rs[k]).astype(np.float64)
        q0, r0 = reference.chol_eqr(a32, z32)
        aq2 = metrics.diagnostics(a32, z32, q0, r0)["a_q2"]
        assert metrics.orth_loss(a32, q) <= max(1e-6, 10 * U32 * aq2), k
        assert metrics.residual_f(z32, q, r) <= 1e-6, k


def test_batch_split_failing_instance_reports_and_stops():
    """A split instance whose Gram is not positive definite reports its pivot in info after the first
    pass and takes no second pass; the other instances, split or not, are solved."""
    insts = make_batch(10, m_lo=100, m_hi=1000, seed=17)
    m, n = 900, 5
    d = np.ones(m)
    d[1] = -1.0
    bad_a = np.diag(d)
    bad_z = np.zeros((m, n), order="F")
    for j in range(n):
        bad_z[j, j] = 1.0
    insts[2] = (bad_a, bad_z)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs, tuning=_split_tuning(500, 3))
    banner("batch split with a failing instance")
    plan.run()
    torch.cuda.synchronize()
    info = to_host(plan.info)
    assert info[2] == variants.chol_info(bad_z.T @ bad_a @ bad_z)[1] == 2
    good = [k for k in range(len(insts)) if k != 2]
    assert np.all(info[good] == 0)
    for k in good:
        a, z = insts[k]
        assert metrics.residual_f(z, to_host(plan.Qs[k]), to_host(plan.Rs[k])) <= 1e-12


def test_batch_split_graph_replays_match_eager():
    insts = make_batch(12, m_lo=200, m_hi=1500, seed=18)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs, tuning=_split_tuning(800, 4))
    plan.run()
    torch.cuda.synchronize()
    eager_q = [q.clone() for q in plan.Qs]
    eager_r = [r.clone() for r in plan.Rs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.run()
    banner("batch split graph replays")
    for rep in range(3):
        for q in plan.Qs:
            q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(plan.info.sum().item()) == 0
        for k in range(len(insts)):
            assert torch.equal(plan.Qs[k], eager_q[k]) and torch.equal(plan.Rs[k], eager_r[k]), (rep, k)


def test_batch_bucket_table_selects_per_class():
    """A table with a different shape per (m bucket, n class): every instance still matches the oracle."""
    insts = make_batch(32, m_lo=200, m_hi=1100, seed=14)
    As, Zs = upload(insts, np.float64)
    d = oqr.default_batch_tuning().to_dict()
    d["shape"] = [[(b + c) % oqr.BATCH_SHAPES for c in range(oqr.BATCH_NCLASSES)] for b in range(oqr.BATCH_MBUCKETS)]
    plan = oqr.BatchPlan(As, Zs, tuning=oqr.BatchTuning.from_dict(d))
    banner("batch mixed shape table")
    plan.run()
    torch.cuda.synchronize()
    check_fp64(insts, plan)


def test_batch_fp32_storage():
    insts = make_batch(24, seed=9, k=(1e2, 1e4))
    As, Zs = upload(insts, np.float32)
    plan = oqr.BatchPlan(As, Zs)
    banner("batch fp32")
    plan.run()
    torch.cuda.synchronize()
    assert np.all(to_host(plan.info) == 0)
    for k, (a, z) in enumerate(insts):
        a32 = a.astype(np.float32).astype(np.float64)     # the oracle sees the rounded inputs
        z32 = z.astype(np.float32).astype(np.float64)
        q, r = to_host(plan.Qs[k]).astype(np.float64), to_host(plan.Rs[k]).astype(np.float64)
        q0, r0 = reference.chol_eqr(a32, z32)
        aq2 = metrics.diagnostics(a32, z32, q0, r0)["a_q2"]
        assert metrics.orth_loss(a32, q) <= max(1e-6, 10 * U32 * aq2), k
        assert metrics.residual_f(z32, q, r) <= 1e-6, k
        assert metrics.r_forward_error(r, r0) <= 1e-5 * max(1.0, np.linalg.cond(r0) * U32 * 1e3), k


def test_batch_matches_per_instance_launches():
    insts = make_batch(12, seed=10)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs)
    plan.run()
    banner("batch vs per-instance")
    for k in range(len(insts)):
        q1, r1 = oqr.cholqr2(As[k], Zs[k])
        n = insts[k][1].shape[1]
        kap = np.linalg.cond(to_host(r1))
        assert metrics.r_forward_error(to_host(plan.Rs[k]), to_host(r1)) <= 10 * n * U * kap
        assert np.abs(to_host(plan.Qs[k]) - to_host(q1)).max() <= 10 * n * U * kap * np.abs(to_host(q1)).max()


def test_failing_instance_does_not_stop_the_batch():
    insts = make_batch(10, seed=11)
    m, n = 200, 5
    d = np.ones(m)
    d[1] = -1.0
    bad_a = np.diag(d)
    bad_z = np.zeros((m, n), order="F")
    for j in range(n):
        bad_z[j, j] = 1.0
    insts[3] = (bad_a, bad_z)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs)
    banner("batch with a failing instance")
    plan.run()
    torch.cuda.synchronize()
    info = to_host(plan.info)
    assert info[3] == variants.chol_info(bad_z.T @ bad_a @ bad_z)[1] == 2
    good = [k for k in range(len(insts)) if k != 3]
    assert np.all(info[good] == 0)
    for k in good:
        a, z = insts[k]
        assert metrics.residual_f(z, to_host(plan.Qs[k]), to_host(plan.Rs[k])) <= 1e-12


def test_malformed_items_are_flagged_and_left_alone():
    """Items outside the entry point's limits (n above 64, m above max_m, lda below m, a null R,
    an A whose leading dimension spans more than 2^31 - 1 bytes) get OQR_BATCH_BAD_ITEM, their
    outputs stay untouched, and every other instance is solved as usual."""
    insts = make_batch(8, seed=13)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs)
    items = (oqr.BatchItem * plan.batch).from_buffer_copy(bytes(plan.items.cpu().numpy()))
    items[1].n = 65
    items[2].m = plan.max_m + 1
    items[4].lda = items[4].m - 1
    items[5].r = None
    items[6].lda = 2 ** 28
    bad = [1, 2, 4, 5, 6]
    plan.items.copy_(torch.frombuffer(bytearray(bytes(items)), dtype=torch.uint8))
    for k in bad:
        plan.Qs[k].fill_(float("nan"))
        plan.Rs[k].fill_(float("nan"))
    banner("batch with malformed items")
    plan.run()
    torch.cuda.synchronize()
    info = to_host(plan.info)
    assert np.all(info[bad] == oqr.OQR_BATCH_BAD_ITEM), info
    for k in bad:
        assert np.all(np.isnan(to_host(plan.Qs[k]))) and np.all(np.isnan(to_host(plan.Rs[k])))
    good = [k for k in range(len(insts)) if k not in bad]
    assert np.all(info[good] == 0), info
    for k in good:
        a, z = insts[k]
        assert metrics.residual_f(z, to_host(plan.Qs[k]), to_host(plan.Rs[k])) <= 1e-12


def test_graph_capture_replays_match_eager():
    """The batched launch captured in a graph: several replays, with eager work and syncs between
    them, each equal bit for bit to the eager result."""
    insts = make_batch(16, seed=12)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs)
    plan.run()                       # eager reference (also primes the device queries)
    torch.cuda.synchronize()
    eager_q = [q.clone() for q in plan.Qs]
    eager_r = [r.clone() for r in plan.Rs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        plan.run()
    banner("graph replays")
    for rep in range(4):
        for q in plan.Qs:
            q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(plan.info.sum().item()) == 0
        for k in range(len(insts)):
            assert torch.equal(plan.Qs[k], eager_q[k]) and torch.equal(plan.Rs[k], eager_r[k]), (rep, k)


def test_autotune_picks_shapes_and_results_hold():
    """BatchPlan.autotune times the four tile shapes on each (m bucket, n class) present and the
    workgroups per compute unit, keeps the fastest; the tuned launch still matches the oracle and
    repeats its bits."""
    insts = make_batch(24, seed=9)
    As, Zs = upload(insts, np.float64)
    plan = oqr.BatchPlan(As, Zs, tuning=oqr.default_batch_tuning())
    banner("batch autotune")
    rep = plan.autotune(reps=2)
    classes = {(oqr.batch_m_bucket(z.shape[0]), oqr.batch_n_class(z.shape[1])) for _, z in insts}
    assert len(rep["classes"]) == len(classes)
    for (b, c) in classes:
        e = rep["classes"][f"m{b}_n{c}"]
        assert set(e["ms"]) == set(oqr.BATCH_SHAPE_NAMES) and all(v > 0 for v in e["ms"].values())
        assert e["shape"] == min(e["ms"], key=e["ms"].get)
        assert oqr.BATCH_SHAPE_NAMES[plan.tuning.shape[b][c]] == e["shape"]
    assert plan.tuning.wg_per_cu == min(rep["wg_per_cu"], key=rep["wg_per_cu"].get)
    plan.run()
    torch.cuda.synchronize()
    check_fp64(insts, plan)
    q1 = [q.clone() for q in plan.Qs]
    plan.run()
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(plan.Qs[k], q1[k])


def test_stored_tuning_table_is_valid():
    """The tuning table checked in beside the library parses into the launch's limits."""
    for dtype in ("f64", "f32"):
        t = oqr.stored_batch_tuning(dtype)
        assert t is not None, dtype
        assert 1 <= t.wg_per_cu <= 3 and t.sort in (0, 1)
        assert all(0 <= t.shape[b][c] < oqr.BATCH_SHAPES
                   for b in range(oqr.BATCH_MBUCKETS) for c in range(oqr.BATCH_NCLASSES))
