"""GPU parity of CHOLQR-A and CholQR2-A (dense and stencil) against the CPU oracle.

Tolerances (derived in the design notes from Theorem 2.1 and the readings of
the paper): residual ||Z - QR||_F/||Z||_F <= 1e-12 for every FP64 path;
orthogonality ||I - Q^T A Q||_2 <= 1e-12 for CholQR2-A (the stable class, loss
c m n u ||A|| ||Q||^2); CHOLQR-A single pass is judged against the same
algorithm's CPU FP64 behaviour (loss within 10x + a floor) because its loss
grows like kappa(A^{1/2} Z)^2; R forward error <= 10 n u kappa(A^{1/2} Z)
against the oracle for the stable variant.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import U, banner, to_dev, to_dev_colmajor, to_host
from golden_data import load as load_golden
from oracle import metrics, reference, variants

pytestmark = pytest.mark.gpu

oqr = pytest.importorskip("paper_1401_5171_amd")


def dense_case(cfg, m, n, ka, kz, seed=0, kind="haar"):
    rng = W.rng_for(cfg, seed, m, n)
    a, _, _ = W.dense_spd(rng, m, ka, kind=kind)
    z = W.tall_skinny(rng, m, n, kz)
    return a, z


def run_dense(alg, a, z, **kw):
    A = to_dev(a)
    Z = to_dev_colmajor(z)
    q, r = getattr(oqr, alg)(A, Z, **kw)
    return to_host(q), to_host(r)


@pytest.mark.parametrize("name", ["random_m10_n3", "random_m24_n6", "case3_m20_n4", "n1_m16"])
def test_cholqr2_matches_golden(name):
    d = load_golden()[name]
    banner(f"golden {name}")
    q, r = run_dense("cholqr2", d["A"], d["Z"])
    kap = np.linalg.cond(d["R"])
    assert metrics.r_forward_error(r, d["R"]) <= 100 * d["n"] * U * kap
    # forward error of Q = Z R^{-1} inherits kappa(R) from the R error
    assert np.abs(q - d["Q"]).max() <= 10 * d["n"] * U * kap * np.abs(d["Q"]).max()
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)


def test_config1_all_fp64_paths():
    """m=500, n=20, kappa(A)=1e4, kappa(Z)=1e3 (the first workload)."""
    rng = W.rng_for(1)
    a, _, _ = W.dense_spd(rng, 500, 1e4)
    z = W.tall_skinny(rng, 500, 20, 1e3)
    q0, r0 = reference.chol_eqr(a, z)
    kap = np.linalg.cond(r0)
    banner("config1 cholqr2")
    q, r = run_dense("cholqr2", a, z)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(a, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * 20 * U * kap
    banner("config1 cholqr")
    q1, r1 = run_dense("cholqr", a, z)
    qc, rc = variants.cholqr(a, z)
    assert metrics.residual_f(z, q1, r1) <= 1e-12
    assert metrics.orth_loss(a, q1) <= 10 * metrics.orth_loss(a, qc) + 1e-13
    assert metrics.r_forward_error(r1, rc) <= 10 * 20 * U * kap


@pytest.mark.parametrize("kz", [1e1, 1e4, 1e7])
def test_config2_shape_kappa_sweep(kz):
    """Second workload's structure (kappa(A) = 1e6, Haar factors) at m = 2048, n = 64."""
    a, z = dense_case(2, 2048, 64, 1e6, kz)
    q0, r0 = reference.chol_eqr(a, z)
    banner(f"config2-shape kz={kz:g}")
    q, r = run_dense("cholqr2", a, z)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(a, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * 64 * U * np.linalg.cond(r0)


@pytest.mark.parametrize("m,n", [(1, 1), (7, 3), (65, 65), (130, 1), (1000, 37), (777, 100), (1531, 129), (600, 256),
                                 (3000, 50), (5003, 130), (257, 129), (2049, 200), (3333, 161), (4133, 255)])
def test_ragged_shapes(m, n):
    """Sizes that leave partial tiles in every kernel (and m = n, n = 1); for 128 < n <= 256 the
    right-looking substitution (partial 16-column tiles, a last block narrower than 32) and the
    all-tiles Gram that adds the product's layers as it loads them."""
    ka = 1e3 if m > 1 else 1.0
    a, z = dense_case(90, m, n, ka, 10.0)
    banner(f"ragged m={m} n={n}")
    q, r = run_dense("cholqr2", a, z)
    q0, r0 = reference.chol_eqr(a, z)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(a, q) <= 1e-12 * max(1.0, metrics.diagnostics(a, z, q0, r0)["a_q2"] / 100)
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0) + 1e-15


@pytest.mark.parametrize("m,n", [(700, 24), (1100, 200)])
def test_in_place_q_aliases_z(m, n):
    a, z = dense_case(91, m, n, 1e4, 1e3)
    A = to_dev(a)
    Z = to_dev_colmajor(z)
    plan = oqr.Plan("cholqr2", A, n)
    import torch
    R = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
    banner(f"in place m={m} n={n}")
    plan.run(Z, Z, R)
    assert int(plan.info.item()) == 0
    q, r = to_host(Z), to_host(R)
    assert metrics.residual_f(z, q, r) <= 1e-12 and metrics.orth_loss(a, q) <= 1e-12


def test_deterministic_bitwise():
    a, z = dense_case(92, 1500, 48, 1e5, 1e4)
    banner("determinism")
    q1, r1 = run_dense("cholqr2", a, z)
    q2, r2 = run_dense("cholqr2", a, z)
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)


def test_info_reports_failed_pivot():
    """A indefinite in the span of Z: the 3rd pivot is negative at any shift the retry rule tries."""
    m, n = 300, 5
    d = np.ones(m)
    d[2] = -1.0
    a = np.diag(d)
    z = np.zeros((m, n), order="F")
    for j in range(n):
        z[j, j] = 1.0
    r_cpu, info_cpu = variants.chol_info(z.T @ a @ z)
    assert info_cpu == 3
    A = to_dev(a)
    plan = oqr.Plan("cholqr", A, n)
    banner("info")
    with pytest.raises(oqr.OQRError) as e:
        plan(to_dev_colmajor(z))
    assert e.value.info == info_cpu


def test_nan_input_reports_first_pivot():
    a, z = dense_case(93, 200, 8, 1e2, 10.0)
    z[5, 0] = np.nan
    with pytest.raises(oqr.OQRError) as e:
        run_dense("cholqr2", a, z)
    assert e.value.info == 1


def test_argument_errors_are_reported():
    a, z = dense_case(94, 100, 4, 10.0, 10.0)
    A = to_dev(a)
    with pytest.raises(ValueError):
        oqr.cholqr2(A, to_dev_colmajor(z[:, :3])[:50])   # shape mismatch caught in the binding
    zz = to_dev_colmajor(np.zeros((100, 300)))
    with pytest.raises(oqr.OQRError) as e:
        oqr.Plan("cholqr2", A, 300)                        # n > 256 unsupported
    del zz


def test_device_check_matches_cpu_metrics():
    a, z = dense_case(95, 900, 30, 1e4, 1e3)
    q, r = reference.chol_eqr(a, z)
    q = q + 1e-9 * np.random.default_rng(0).standard_normal(q.shape)   # make the errors visible
    A = to_dev(a)
    banner("check")
    orth_f, res_f = oqr.check(A, to_dev_colmajor(z), to_dev_colmajor(q), to_dev_colmajor(r))
    g = q.T @ a @ q
    assert abs(orth_f - np.linalg.norm(g - np.eye(30))) <= 1e-6 * orth_f
    assert abs(res_f - metrics.residual_f(z, q, r)) <= 1e-6 * res_f


# ---- stencil operator --------------------------------------------------------------------------

@pytest.mark.parametrize("grid,n", [((16, 12, 10), 32), ((33, 17, 9), 45), ((40, 40, 20), 128)])
def test_stencil_cholqr2_fp64(grid, n):
    st = W.laplacian7(*grid)
    z = W.gaussian_scaled(W.rng_for(3, 0, *grid), st.m, n, 1e4)
    q0, r0 = reference.stencil_eqr(st, z)
    banner(f"stencil fp64 grid={grid} n={n}")
    q, r = (to_host(x) for x in oqr.cholqr2(oqr.Stencil7(*grid, st.center, st.off), to_dev_colmajor(z)))
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)


@pytest.mark.parametrize("n", [40, 100])
def test_stencil_large_grid_persistent_paths(n):
    """m = 135135 rows (a ragged last 64-row tile, more than 2000 tiles): the z-marching stencil, the
    all-tiles Gram and the persistent substitution with R held in registers."""
    grid = (65, 63, 33)
    st = W.laplacian7(*grid)
    z = W.gaussian_scaled(W.rng_for(3, 1, *grid), st.m, n, 1e4)
    q0, r0 = reference.stencil_eqr(st, z)
    banner(f"stencil large grid={grid} n={n}")
    op = oqr.Stencil7(*grid, st.center, st.off)
    q, r = (to_host(x) for x in oqr.cholqr2(op, to_dev_colmajor(z)))
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)
    q1, r1 = (to_host(x) for x in oqr.cholqr2(op, to_dev_colmajor(z), pass1="bf16x3"))
    assert metrics.residual_f(z, q1, r1) <= 1e-12
    assert metrics.orth_loss(st, q1) <= 1e-12


def test_stencil_single_pass_reaches_fp64_on_column_scaled_z():
    """Column scaling alone (kappa(Z) from diag(s)) is harmless to CHOLQR: one FP64 pass suffices."""
    grid, n = (24, 24, 12), 64
    st = W.laplacian7(*grid)
    z = W.gaussian_scaled(W.rng_for(3, 1), st.m, n, 1e4)
    banner("stencil single pass")
    q, r = (to_host(x) for x in oqr.cholqr(oqr.Stencil7(*grid, st.center, st.off), to_dev_colmajor(z)))
    qc, rc = variants.cholqr(st, z)
    assert metrics.orth_loss(st, q) <= 10 * metrics.orth_loss(st, qc) + 1e-14
    assert metrics.residual_f(z, q, r) <= 1e-12


# ---- mixed precision ---------------------------------------------------------------------------

@pytest.mark.parametrize("pass1", ["bf16x2", "bf16x3"])
def test_mixed_pass1_then_fp64_reaches_fp64_orthogonality(pass1):
    """Split-bfloat16 A Z in pass 1, FP64 pass 2: orthogonality <= 1e-12, residual <= 1e-12."""
    a, z = dense_case(2, 2048, 64, 1e6, 1e4, seed=5, kind="butterfly")
    banner(f"mixed {pass1}+fp64")
    q, r = run_dense("cholqr2", a, z, pass1=pass1, pass2="fp64")
    q0, r0 = reference.chol_eqr(a, z)
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(a, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * 64 * U * np.linalg.cond(r0)


def test_mixed_first_pass_matches_emulated_error_level():
    """One BF16x3 pass: the GPU's loss of orthogonality sits within 10x of the CPU emulation
    of the same arithmetic (level, not bits: accumulation order differs)."""
    from oracle import mixed
    a, z = dense_case(2, 1024, 32, 1e4, 1e4, seed=6, kind="butterfly")
    qe, re, info, s = mixed.cholqr_pass(a, z, "bf16x3", shift_c=1.0)
    assert info == 0
    banner("mixed single pass vs emulation")
    q, r = run_dense("cholqr", a, z, prec="bf16x3", shift_c=1.0)
    le, lg = metrics.orth_loss(a, qe), metrics.orth_loss(a, q)
    assert le / 10 <= lg <= 10 * le, (le, lg)
    assert metrics.residual_f(z, q, r) <= 1e-12       # FP64 substitution keeps the residual at FP64 level


@pytest.mark.parametrize("m,n,prec", [(4096, 256, "bf16x3"), (3001, 200, "bf16x3"), (2113, 129, "bf16x2")])
def test_mixed_wide_n(m, n, prec):
    """n > 128 takes the 512-thread split product over K-step-tiled slices of Z, the diagonal blocks as a
    layer of their own and the Gram adding the layers as it loads them: one split pass at the emulated
    error level, and split + FP64 CholQR2 at FP64 orthogonality (ragged m and n included)."""
    from oracle import mixed
    a, z = dense_case(2, m, n, 1e4, 1e3, seed=8, kind="butterfly")
    banner(f"mixed wide n m={m} n={n} {prec}")
    qe, re, info, s = mixed.cholqr_pass(a, z, prec, shift_c=1.0)
    assert info == 0
    q, r = run_dense("cholqr", a, z, prec=prec, shift_c=1.0)
    le, lg = metrics.orth_loss(a, qe), metrics.orth_loss(a, q)
    assert le / 10 <= lg <= 10 * le, (le, lg)
    assert metrics.residual_f(z, q, r) <= 1e-12
    q2, r2 = run_dense("cholqr2", a, z, pass1=prec, pass2="fp64")
    q0, r0 = reference.chol_eqr(a, z)
    assert metrics.residual_f(z, q2, r2) <= 1e-12
    assert metrics.orth_loss(a, q2) <= 1e-12
    assert metrics.r_forward_error(r2, r0) <= 10 * n * U * np.linalg.cond(r0)


def test_fully_mixed_cholqr2_meets_mixed_tolerance():
    """Both passes BF16x3: orthogonality <= max(1e-6, 10 u_p ||A|| ||Q||^2) with u_p = 2^-24."""
    a, z = dense_case(2, 1500, 40, 1e5, 1e3, seed=7, kind="butterfly")
    q0, r0 = reference.chol_eqr(a, z)
    aq2 = metrics.diagnostics(a, z, q0, r0)["a_q2"]
    banner("fully mixed")
    q, r = run_dense("cholqr2", a, z, pass1="bf16x3", pass2="bf16x3")
    assert metrics.orth_loss(a, q) <= max(1e-6, 10 * 2.0 ** -24 * aq2)
    assert metrics.residual_f(z, q, r) <= 1e-12


@pytest.mark.parametrize("pass1", ["bf16x2", "bf16x3"])
def test_stencil_mixed_gram_then_fp64(pass1):
    grid, n = (32, 32, 16), 64
    st = W.laplacian7(*grid)
    rng = W.rng_for(3, 2)
    z = W.tall_skinny(rng, st.m, n, 1e4)     # Haar-mixed Z (the stress variant)
    q0, r0 = reference.stencil_eqr(st, z)
    banner(f"stencil mixed {pass1}")
    q, r = (to_host(x) for x in oqr.cholqr2(oqr.Stencil7(*grid, st.center, st.off), to_dev_colmajor(z),
                                             pass1=pass1, pass2="fp64"))
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)


@pytest.mark.parametrize("pass1,n,grid", [("bf16x3", 64, (33, 17, 20)), ("bf16x2", 100, (20, 24, 9))])
def test_stencil_fused_split_pass_matches_emulated_error_level(pass1, n, grid):
    """One split-bfloat16 CholQR pass on the stencil (A Z formed inside the split Gram kernel): the GPU's
    loss of orthogonality sits within 10x of the CPU emulation of the same arithmetic (exact FP64 stencil,
    split operands, FP32 sums over 256-row tiles). Level, not bits: the GPU's K tiles are plane regions,
    the emulation's consecutive rows. Ragged regions (nx not a multiple of 16), n = 64 and 100."""
    from oracle import mixed
    st = W.laplacian7(*grid)
    z = W.tall_skinny(W.rng_for(3, 4, *grid), st.m, n, 1e3)
    qe, re, info, s = mixed.cholqr_pass(st, z, pass1, shift_c=1.0)
    assert info == 0
    banner(f"stencil fused split pass {pass1} grid={grid} n={n}")
    q, r = (to_host(x) for x in oqr.cholqr(oqr.Stencil7(*grid, st.center, st.off), to_dev_colmajor(z),
                                            prec=pass1, shift_c=1.0))
    le, lg = metrics.orth_loss(st, qe), metrics.orth_loss(st, q)
    assert le / 10 <= lg <= 10 * le, (le, lg)
    assert metrics.residual_f(z, q, r) <= 1e-12


@pytest.mark.parametrize("grid,n,pass1,pad", [
    ((1, 1, 1), 1, "fp64", 0),        # a single grid point
    ((5, 3, 1), 3, "fp64", 0),        # one plane; 16-point regions straddle lines of 5
    ((1, 7, 6), 5, "bf16x3", 0),      # lines of one point: no x-neighbours
    ((9, 1, 17), 65, "fp64", 5),      # ny = 1; one column in the second 64-column block; ld = m + 5
    ((6, 5, 40), 128, "bf16x2", 3),   # n = 128, ld = m + 3
    ((256, 192, 2), 8, "fp64", 0),    # 3072 plane regions: workgroups march several regions
    ((256, 192, 2), 70, "bf16x3", 0),
])
def test_stencil_fused_gram_edge_shapes(grid, n, pass1, pad):
    """The fused stencil Gram (FP64 and split) on degenerate grids and a padded leading dimension of Z:
    CholQR2 against the oracle's whitened Householder QR."""
    import torch
    st = W.laplacian7(*grid)
    z = W.tall_skinny(W.rng_for(3, 5, *grid), st.m, n, 1e2)
    q0, r0 = reference.stencil_eqr(st, z)
    banner(f"stencil fused edge grid={grid} n={n} pass1={pass1} pad={pad}")
    zd = torch.empty(n, st.m + pad, dtype=torch.float64, device="cuda").t()[: st.m]
    zd.copy_(torch.from_numpy(np.asarray(z, dtype=np.float64)))
    q, r = (to_host(x) for x in oqr.cholqr2(oqr.Stencil7(*grid, st.center, st.off), zd, pass1=pass1, pass2="fp64"))
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * max(n, 2) * U * np.linalg.cond(r0)


@pytest.mark.parametrize("n,ld,pass1", [(150, None, "fp64"), (150, None, "bf16x3"), (2, 4_400_000, "fp64"),
                                        (2, 4_400_000, "bf16x2")])
def test_stencil_unfused_fallbacks(n, ld, pass1):
    """The stencil paths that do not fuse A Z into the Gram: n > 128 (apply + tile Gram), and a leading
    dimension of Z too large for 32-bit offsets inside a 64-column block (apply + all-tiles Gram)."""
    import torch
    grid = (16, 12, 10)
    st = W.laplacian7(*grid)
    z = W.tall_skinny(W.rng_for(3, 6, n), st.m, n, 1e2)
    q0, r0 = reference.stencil_eqr(st, z)
    banner(f"stencil unfused n={n} ld={ld} pass1={pass1}")
    if ld is None:
        zd = to_dev_colmajor(z)
    else:
        zd = torch.empty(n, ld, dtype=torch.float64, device="cuda").t()[: st.m]
        zd.copy_(torch.from_numpy(np.asarray(z, dtype=np.float64)))
    q, r = (to_host(x) for x in oqr.cholqr2(oqr.Stencil7(*grid, st.center, st.off), zd, pass1=pass1, pass2="fp64"))
    assert metrics.residual_f(z, q, r) <= 1e-12
    assert metrics.orth_loss(st, q) <= 1e-12
    assert metrics.r_forward_error(r, r0) <= 10 * n * U * np.linalg.cond(r0)
