"""The seeded input generators (Section 7's constructions): spectra, orthogonality of the random
factors, and agreement of the host and torch builds of the same matrices."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")


def test_logspace_runs_from_one_to_kappa():
    d = W.logspace_to(50, 1e6)
    assert d[0] == 1.0 and abs(d[-1] / 1e6 - 1) < 1e-13 and np.all(np.diff(d) > 0)
    assert W.logspace_to(1, 1e6).tolist() == [1.0]


def test_haar_and_butterfly_are_orthogonal():
    rng = W.rng_for(90)
    v = W.haar(rng, 120, 120)
    assert np.linalg.norm(v.T @ v - np.eye(120)) < 1e-13
    b = W.butterfly(rng, 300, block=64)
    vb = b.dense()
    assert np.linalg.norm(vb.T @ vb - np.eye(300)) < 1e-13
    x = rng.standard_normal((300, 3))
    assert np.allclose(b.apply(x), vb @ x, rtol=0, atol=1e-13)
    xt = torch.from_numpy(x)
    assert np.allclose(b.apply_torch(xt).numpy(), vb @ x, rtol=0, atol=1e-13)


def test_tall_skinny_has_the_requested_singular_values():
    z = W.tall_skinny(W.rng_for(91), 200, 12, 1e5)
    s = np.linalg.svd(z, compute_uv=False)
    assert np.allclose(np.sort(s), W.logspace_to(12, 1e5), rtol=1e-12)


def test_torch_and_numpy_spd_builds_agree():
    rng = W.rng_for(92)
    b = W.butterfly(rng, 200, block=64)
    d = W.logspace_to(200, 1e4)
    a = W.spd_from_eigs(b, d)
    at = W.spd_from_eigs_torch(b, d, "cpu").numpy()
    assert np.array_equal(at, at.T)
    assert np.abs(a - at).max() <= 1e-12 * np.abs(a).max()
    assert np.allclose(np.linalg.eigvalsh(at), d, rtol=1e-9)


def test_batch_instance_device_matches_host_instance():
    inst = W.BatchInstance(5, 150, 16, 1e3)
    a, z = W.batch_instance(inst)
    at, zt = W.batch_instance_device(inst, "cpu")
    assert tuple(zt.shape) == (150, 16) and zt.stride() == (1, 150)
    assert np.array_equal(zt.numpy(), z)
    assert np.abs(at.numpy() - a).max() <= 1e-12 * np.abs(a).max()


def test_batch_plan_ranges():
    plan = W.batch_plan(400)
    ms = np.array([p.m for p in plan])
    ns = {p.n for p in plan}
    ks = np.array([p.kappa for p in plan])
    assert ms.min() >= 256 and ms.max() <= 4096 and ns == {8, 16, 32, 64}
    assert ks.min() >= 1e2 and ks.max() <= 1e8
    assert [p.m for p in W.batch_plan(400)] == ms.tolist()      # seeded: the same sizes every time
