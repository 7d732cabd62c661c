#!/usr/bin/env python3
"""Oblique-QR benchmark on one MI355X: mixed-precision vs FP64 CholQR2-A.

Default workload: dense SPD A, m = 32768, n = 256, kappa(A) = 1e8 (log-spaced
eigenvalues, dense random orthogonal eigenvectors), Z = U diag(s) W^T with
kappa(Z) = 1e5 (Haar factors).  One step = one CholQR2-A factorisation of Z:
pass 1 with A Z on split-bfloat16 MFMA (by default two slices, hi = bf16(x)
and lo = bf16(x - hi), products hi*hi + hi*lo + lo*hi; --pass1 bf16x3 for
three slices), FP32 accumulation inside K tiles, FP64 across them, FP64
Gram/Cholesky/substitution; pass 2 all FP64.  The same step in all-FP64 is
timed beside it.

Throughput uses the paper's normalised flop count 2 m^2 n + 2 m n^2 for one
factorisation (Section 8), whatever the algorithm executes.  Inputs are
resident in HBM before the timed region; the timed region is K back-to-back
steps bracketed by device synchronisation.  The roofline entry is the
dominant kernel (the FP64 A-times-Q1 product of pass 2), its average launch
time taken from HIP events recorded around each launch inside the timed
region.  The CPU baseline times the CPU oracle (CHOL-EQR, Algorithm 3) on the
leading m' x m' sub-problem.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dense32768|dense8192|stencil|tridiag|batch|small500]

The batch workload (4096 independent instances, m log-uniform in [256, 4096], n in {8, 16, 32, 64},
kappa(A_i) log-uniform in [1e2, 1e8], Gaussian Z_i) times one persistent launch of the batched
FP64 CholQR2-A over all instances, beside the same factorisations launched one instance at a time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "oblique-QR GFLOP/s & % roofline, mixed vs FP64 CholQR2-A at orth loss ≤1e-12"
PEAK = {"fp64": 78.6e12, "bf16": 2.5e15, "hbm": 8.0e12}
# L2-miss bytes per launch of the dominant kernel (an upper bound on its HBM bytes: the MALL serves part of
# them), from two rocprofv3 counter runs of this script (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) scaled by what the same counters read for a 1 GiB copy
# (--workload copycal: FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Only for the kernel build they were taken
# on; workloads without an entry report null.
TRAFFIC = {
    ("dense32768", "gemm_f64"): (8529916.3 * 2.0 + 131084.7 * 1.0) * 1024,
    ("stencil", "gram"): (1001810.9 * 2.0 + 73731.6 * 1.0) * 1024,
}


def upper_product_flops(m, n, bm=64, diag=False):
    """Algorithmic flops of the FP64 product over the strictly upper block triangle of a symmetric A
    (row tiles of bm rows; tile t multiplies its rows of A over K in [bm (t + 1), m) by Z), or with diag
    over the upper block triangle including the diagonal blocks (K from bm t: the FP64 pass's
    W' = (U + D/2) Z, whose diagonal blocks take the place of the separate D Z product)."""
    total = 0
    for t0 in range(0, m, bm):
        rows = min(bm, m - t0)
        total += 2 * rows * n * (m - min(m, t0 + (0 if diag else bm)))
    return float(total)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="dense32768",
                   choices=["dense32768", "dense8192", "stencil", "tridiag", "batch", "small500", "copycal"])
    p.add_argument("--batch-count", type=int, default=4096)
    p.add_argument("--batch-dtype", default="f64", choices=["f64", "f32"], help="storage type of the batch")
    p.add_argument("--retune", action="store_true",
                   help="batch: autotune the tile shapes on this batch instead of using the stored table")
    p.add_argument("--pass1", default=None, choices=["fp64", "bf16x2", "bf16x3"],
                   help="precision of pass 1 of the mixed schedule (default bf16x2: hi/lo split)")
    p.add_argument("--cpu-sample", type=int, default=8192, help="m' of the CPU oracle sample (0 = skip)")
    p.add_argument("--no-others", action="store_true",
                   help="default workload only: skip the stencil and batch summaries added to its line")
    return p.parse_args()


def make_inputs(wl, torch):
    import numpy as np
    import workloads as W
    import paper_1401_5171_amd as oqr
    dev = torch.device("cuda", 0)
    if wl in ("dense32768", "dense8192"):
        m = 32768 if wl == "dense32768" else 8192
        cfg = 4 if m == 32768 else 2
        n, ka, kz = (256, 1e8, 1e5) if m == 32768 else (64, 1e6, 1e4)
        rng = W.rng_for(cfg, 0)
        t = time.time()
        A, _, _ = W.dense_spd_device(rng, m, ka, dev)
        z = W.tall_skinny(rng, m, n, kz)
        log(f"generated A ({m}x{m}) on the device and Z in {time.time() - t:.1f}s")
        Z = torch.from_numpy(np.ascontiguousarray(z.T)).to(dev).t()
        desc = dict(workload=f"dense SPD A m={m} n={n} kappa(A)={ka:g} kappa(Z)={kz:g}", m=m, n=n,
                    kappa_a=ka, kappa_z=kz, operator="dense", eigenvectors="butterfly-Haar",
                    seeds=f"SeedSequence([15171, {cfg}, 0])")
        flops = 2.0 * m * m * n + 2.0 * m * n * n
        return A, Z, z, m, n, desc, flops, "gemm_f64", upper_product_flops(m, n, diag=True)
    if wl == "tridiag":
        m, n = 100000, 64
        t = W.laplacian1d(m, 1e-3)
        z = W.tall_skinny(W.rng_for(6, 0), m, n, 1e3)
        Z = torch.from_numpy(np.ascontiguousarray(z.T)).to(dev).t()
        A = oqr.Tridiag(t.diag, t.sub, device=dev)
        A.host = t
        desc = dict(workload=f"tridiagonal A (1D Dirichlet Laplacian + 1e-3 I) m={m} n={n} kappa(Z)=1e3",
                    m=m, n=n, operator="tridiag")
        return A, Z, z, m, n, desc, 2.0 * m * n * n, "trsm", 1.0 * m * n * n
    nx, ny, nz, n = 128, 128, 64, 128
    st = W.laplacian7(nx, ny, nz)
    rng = W.rng_for(3, 0)
    z = W.gaussian_scaled(rng, st.m, n, 1e4)
    Z = torch.from_numpy(np.ascontiguousarray(z.T)).to(dev).t()
    A = oqr.Stencil7(nx, ny, nz, st.center, st.off)
    m = st.m
    desc = dict(workload=f"7-point Laplacian+1e-3 I on {nx}x{ny}x{nz} (m={m}) n={n} kappa(Z)=1e4 column-scaled",
                m=m, n=n, operator="stencil7")
    return A, Z, z, m, n, desc, 2.0 * m * n * n, "gram", 1.0 * m * n * n


def symm_pass_flops(m, n, bm=64):
    """Flops one dense CholQR pass must execute when it exploits A = A^T the way the library does:
    W_off = U Z over the strictly upper blocks of A (row tiles of bm), W_sym = W_off + D Z over the
    diagonal blocks, and the upper triangle of G = Z^T W_sym + W_off^T Z (two products of m n^2 each)."""
    return upper_product_flops(m, n, bm) + 2.0 * n * sum(min(bm, m - t) ** 2 for t in range(0, m, bm)) \
        + 2.0 * m * n * n


def schedule_roofline(kind, m, n, pass_precs, ms):
    """Roofline of a whole CholQR2 schedule: T_roof = sum over passes of max(B / HBM peak, sum over steps
    of F_step / peak of the step's precision), frac = T_roof / measured.  Per pass: dense, the operator
    product and the Gram as the symmetric schedule executes them (symm_pass_flops: A read in its upper
    block triangle, about m^2 n + 2 m n^2 flops instead of the 2 m^2 n + m n^2 of a full product);
    stencil 13 m n (the matrix-free apply, FP64 vector work) + m n^2 (upper triangle of the Gram);
    tridiagonal 5 m n + m n^2; then n^3 / 3 (Cholesky) + m n^2 (substitution), always FP64.  Products and
    Gram run at the bf16 peak in a split pass, FP64 otherwise (the extra slice products are overhead, not
    counted).  B = unique A bytes 8 m (m + 1) / 2 (dense) or 16 m (tridiagonal) + 3 x 8 m n (Z read, Z
    read again by the substitution, Q written).  Every count is work the schedule cannot avoid, so
    frac <= 1."""
    a_bytes = {"dense": 8.0 * m * (m + 1) / 2, "stencil": 0.0, "tridiag": 16.0 * m}[kind]
    t = 0.0
    for prec in pass_precs:
        peak12 = PEAK["bf16"] if prec != "fp64" else PEAK["fp64"]
        if kind == "dense":
            t_mx = symm_pass_flops(m, n) / peak12
        else:
            apply = 13.0 * m * n if kind == "stencil" else 5.0 * m * n
            t_mx = apply / PEAK["fp64"] + m * n * n / peak12
        t_mx += (n ** 3 / 3 + m * n * n) / PEAK["fp64"]
        t += max((a_bytes + 3 * 8.0 * m * n) / PEAK["hbm"], t_mx)
    return {"t_roof_ms": round(t * 1e3, 4), "measured_ms": round(ms, 4), "frac": round(t * 1e3 / ms, 4)}


def time_steps(plan, Z, Q, R, steps, torch, kernel):
    import paper_1401_5171_amd as oqr
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with oqr.KernelTimer(kernel) as kt:
        for _ in range(steps):
            plan.run(Z, Q, R)
        torch.cuda.synchronize()
    t1 = time.perf_counter()
    if int(plan.info.item()) != 0:
        raise RuntimeError(f"numerical failure in the timed region: info={int(plan.info.item())}")
    return (t1 - t0) / steps, kt.avg_ms, kt.count


def breakdown(plan, Z, Q, R, torch):
    import paper_1401_5171_amd as oqr
    out = {}
    for k in ("split_z", "gemm_split", "gemm_f64", "symm_diag", "stencil", "gram", "chol", "trsm"):
        with oqr.KernelTimer(k) as kt:
            plan.run(Z, Q, R)
            torch.cuda.synchronize()
        if kt.count:
            out[k] = round(kt.total_ms, 4)
    return out


def time_variants(A, Z, m, n, flops, torch, reps=3):
    """Every algorithm behind the ABI on the same input (the paper's performance comparison):
    ms per factorisation (best of `reps`), GFLOP/s at the normalised count, orthogonality (F)."""
    import paper_1401_5171_amd as oqr
    out = {}
    specs = [("cholqr", "cholqr", {}), ("cholqr2", "cholqr2", {}), ("pre_cholqr", "pre_cholqr", {}),
             ("chol_eqr", "chol_a", {}), ("cgs", "gs", {"gs_variant": "cgs"}), ("cgs2", "gs", {"gs_variant": "cgs2"}),
             ("mgs_row", "gs", {"gs_variant": "mgs_row"}), ("mgs_col", "gs", {"gs_variant": "mgs_col"})]
    for name, alg, kw in specs:
        plan = oqr.Plan(alg, A, n, **kw)
        Q = torch.empty(n, m, dtype=torch.float64, device="cuda").t()
        R = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
        plan.run(Z, Q, R)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            plan.run(Z, Q, R)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        orth, _ = oqr.check(A, Z, Q, R)
        out[name] = {"ms": round(best * 1e3, 3), "gflops": round(flops / best / 1e9, 2), "orth_loss_fro": orth,
                     "info": int(plan.info.item())}
        log(f"variant {name}: {best * 1e3:.3f} ms, orth {orth:.2e}")
    return out


def cpu_baseline(A, z, n, ms, torch):
    """CPU oracle (CHOL-EQR) on the leading ms x ms block of A and the first ms rows of Z."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import reference
    if hasattr(A, "host"):
        t = time.perf_counter()
        reference.tridiag_eqr(A.host, np.asfortranarray(z))
        dt = time.perf_counter() - t
        f = 2.0 * A.m * n * n
        sample = f"tridiag_eqr (banded CHOL-EQR) on the whole problem, m={A.m}, n={n}"
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        return {"value": round(f / dt / 1e9, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
                "sample": sample, "seconds": round(dt, 3)}
    if hasattr(A, "nx"):
        from oracle import stencil as ost
        import workloads as W
        nz_s = max(1, ms // (A.nx * A.ny))
        st = W.Stencil7(A.nx, A.ny, nz_s, A.center, A.off)
        zs = np.asfortranarray(z[: st.m])
        t = time.perf_counter()
        reference.stencil_eqr(st, zs)
        dt = time.perf_counter() - t
        f = 2.0 * st.m * n * n
        sample = f"stencil_eqr (DST route) on a {A.nx}x{A.ny}x{nz_s} grid (m'={st.m}), n={n}"
    else:
        a = A[:ms, :ms].cpu().numpy()
        zs = np.asfortranarray(z[:ms])
        t = time.perf_counter()
        reference.chol_eqr(a, zs)
        dt = time.perf_counter() - t
        f = 2.0 * ms * ms * n + 2.0 * ms * n * n
        sample = f"chol_eqr on the leading {ms}x{ms} block of A and first {ms} rows of Z, n={n}"
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": round(f / dt / 1e9, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": sample, "seconds": round(dt, 3)}


def run_batch(args, torch, oqr, per_instance=True):
    """Batched FP64 CholQR2-A over the synthetic batch (see the module docstring)."""
    import numpy as np
    import workloads as W
    dev = torch.device("cuda", 0)
    dt = torch.float64 if args.batch_dtype == "f64" else torch.float32
    sizes = W.batch_plan(args.batch_count)
    t = time.time()
    As, Zs = [], []
    for k, p in enumerate(sizes):
        a, z = W.batch_instance_device(p, dev, dt)
        As.append(a)
        Zs.append(z)
        if (k + 1) % 512 == 0:
            log(f"generated {k + 1}/{len(sizes)} instances ({time.time() - t:.1f}s)")
    torch.cuda.synchronize()
    ms = np.array([p.m for p in sizes], dtype=np.float64)
    ns = np.array([p.n for p in sizes], dtype=np.float64)
    flops = float(np.sum(2 * ms * ms * ns + 2 * ms * ns * ns))                  # paper normalisation
    esize = 8 if dt == torch.float64 else 4
    # executed per pass: row block b (128 rows from r0) times A's columns [r0, m) (the kernel reads the
    # upper block triangle of the symmetric A), X_b^T W_b for the diagonal and the right part, the
    # Cholesky and the substitution; bytes: that part of A, and Z / X / Q (m n each)
    alg_flops = alg_bytes = 0.0
    for p in sizes:
        m_, n_ = p.m, p.n
        for r0 in range(0, m_, 128):
            rows = min(128, m_ - r0)
            alg_flops += 2 * (2 * rows * n_ * (m_ - r0) + 2 * rows * n_ * n_ * (2 if r0 + 128 < m_ else 1))
            alg_bytes += 2 * esize * rows * (m_ - r0)
        alg_flops += 2 * (n_ ** 3 / 3 + m_ * n_ * n_)
        alg_bytes += 2 * 3 * esize * m_ * n_
    log(f"batch: {len(sizes)} instances, sum A = {np.sum(ms * ms) * esize / 1e9:.1f} GB, {flops:.3e} flops")
    bp = oqr.BatchPlan(As, Zs)             # the tuning table checked in beside the library
    tune_report = None
    if args.retune:
        tune_report = bp.autotune(reps=3)
        log(f"autotune: {json.dumps(tune_report)}")
    tuning = bp.tuning.to_dict()
    for _ in range(args.warmup):
        bp.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with oqr.KernelTimer("batch") as kt:
        for _ in range(args.steps):
            bp.run()
        torch.cuda.synchronize()
    step = (time.perf_counter() - t0) / args.steps
    info = bp.info.cpu().numpy()
    if np.any(info != 0):
        raise RuntimeError(f"numerical failure in {int(np.sum(info != 0))} instances")
    # accuracy on a stratified sample (every 64th instance), computed on the device in FP64
    worst_o = worst_r = 0.0
    for k in range(0, len(sizes), 64):
        a, z, q, r = (x.double() for x in (As[k], Zs[k], bp.Qs[k], bp.Rs[k]))
        o, rr = oqr.check(a, z, q, r)
        worst_o, worst_r = max(worst_o, o), max(worst_r, rr)
    line_extra = {}
    if dt == torch.float64 and per_instance:
        # the same factorisations, one instance per call (each call launches its own kernels)
        plans = [oqr.Plan("cholqr2", As[k], sizes[k].n) for k in range(len(sizes))]
        outs = [(torch.empty(p.n, p.m, dtype=dt, device=dev).t(), torch.empty(p.n, p.n, dtype=dt, device=dev).t())
                for p in sizes]
        for k, pl in enumerate(plans):
            pl.run(Zs[k], *outs[k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, pl in enumerate(plans):
            pl.run(Zs[k], *outs[k])
        torch.cuda.synchronize()
        per = time.perf_counter() - t0
        line_extra["per_instance_launches"] = {"ms_per_step": round(per * 1e3, 3),
                                               "value": round(flops / per / 1e9, 2),
                                               "batched_speedup": round(per / step, 3)}
        log(f"per-instance launches: {per * 1e3:.2f} ms")
        del plans, outs
    kms = kt.avg_ms
    kname = f"batch_kernel<{'double' if esize == 8 else 'float'}> (tuned tile shapes)"
    # the bound is the resource whose peak needs longer for the launch's algorithmic work
    if alg_bytes / PEAK["hbm"] >= alg_flops / PEAK["fp64"]:
        roof = {"bound": "hbm", "kernel": kname, "achieved": round(alg_bytes / (kms * 1e-3) / 1e9, 1),
                "peak": PEAK["hbm"] / 1e9, "unit": "GB/s", "frac": round(alg_bytes / (kms * 1e-3) / PEAK["hbm"], 4)}
    else:
        roof = {"bound": "mfma", "kernel": kname, "achieved": round(alg_flops / (kms * 1e-3) / 1e12, 3),
                "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s", "frac": round(alg_flops / (kms * 1e-3) / PEAK["fp64"], 4)}
    roof.update({"traffic": None, "per_launch_flops": alg_flops, "per_launch_bytes": alg_bytes,
                 "avg_launch_ms": round(kms, 4),
                 "fp64_mfma_frac": round(alg_flops / (kms * 1e-3) / PEAK["fp64"], 4),
                 "hbm_frac": round(alg_bytes / (kms * 1e-3) / PEAK["hbm"], 4)})
    line = {
        "metric": METRIC, "value": round(flops / step / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if esize == 8 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(sizes)} CholQR2-A instances, m in [256, 4096] log-uniform, "
                               f"n in {{8,16,32,64}}, kappa(A) in [1e2, 1e8], {args.batch_dtype} storage",
                   "count": len(sizes), "flops_per_step": flops, "flop_count": "sum of 2m^2n+2mn^2"},
        "orth_loss_fro_max_sampled": worst_o, "residual_fro_max_sampled": worst_r,
        "tuning": tuning, "autotune": tune_report,
        "roofline": roof, "cpu_baseline": None,
    }
    line.update(line_extra)
    if args.cpu_sample:
        line["cpu_baseline"] = cpu_baseline_batch(As, Zs, sizes, budget_s=12.0)
    del bp, As, Zs
    print(json.dumps(line), flush=True)


def cpu_baseline_batch(As, Zs, sizes, budget_s):
    """CPU oracle (CHOL-EQR) on instances taken every 16th through the batch until the budget is spent."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import reference
    f = dt = 0.0
    done = 0
    for k in range(0, len(sizes), 16):
        a = As[k].double().cpu().numpy()
        z = np.asfortranarray(Zs[k].double().cpu().numpy())
        t = time.perf_counter()
        reference.chol_eqr(a, z)
        dt += time.perf_counter() - t
        f += 2.0 * a.shape[0] ** 2 * z.shape[1] + 2.0 * a.shape[0] * z.shape[1] ** 2
        done += 1
        if dt > budget_s:
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": round(f / dt / 1e9, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"chol_eqr on {done} instances (every 16th of the batch)", "seconds": round(dt, 3)}


def run_copycal(torch):
    """Calibration for HBM counters: three copies of 1 GiB (FP64), so that FETCH_SIZE / WRITE_SIZE
    per dispatch can be compared with the 1 GiB each copy reads and writes."""
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    print(json.dumps({"metric": "copy calibration", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "ms_per_copy": round(dt * 1e3, 4), "GBs": round(2 * nbytes / dt / 1e9, 1)}), flush=True)


def run_small(args, torch, oqr):
    """The smallest workload of the paper's tables: dense A, m = 500 (Haar eigenvectors, kappa(A) = 1e4),
    Z with kappa(Z) = 1e3, n = 20, every variant in FP64.  About 1e7 flops: launch- and latency-bound,
    so the line reports the latency of one factorisation per variant (host call to completion, min and
    median of `steps`) and no roofline fraction."""
    import numpy as np
    import workloads as W
    rng = W.rng_for(1)
    m, n = 500, 20
    a, _, _ = W.dense_spd(rng, m, 1e4)
    z = W.tall_skinny(rng, m, n, 1e3)
    A = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Z = torch.from_numpy(np.ascontiguousarray(z.T)).cuda().t()
    flops = 2.0 * m * m * n + 2.0 * m * n * n
    specs = [("cholqr", "cholqr", {}), ("cholqr2", "cholqr2", {}), ("pre_cholqr", "pre_cholqr", {}),
             ("chol_eqr", "chol_a", {}), ("eqr_syev", "eig_a", {}), ("cgs", "gs", {"gs_variant": "cgs"}),
             ("cgs2", "gs", {"gs_variant": "cgs2"}), ("mgs_row", "gs", {"gs_variant": "mgs_row"}),
             ("mgs_col", "gs", {"gs_variant": "mgs_col"})]
    out = {}
    for name, alg, kw in specs:
        plan = oqr.Plan(alg, A, n, **kw)
        Q = torch.empty(n, m, dtype=torch.float64, device="cuda").t()
        R = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
        for _ in range(max(args.warmup, 1)):
            plan.run(Z, Q, R)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            plan.run(Z, Q, R)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        orth, res = oqr.check(A, Z, Q, R)
        out[name] = {"us_min": round(min(ts) * 1e6, 1), "us_median": round(float(np.median(ts)) * 1e6, 1),
                     "orth_loss_fro": orth, "residual_fro": res, "info": int(plan.info.item())}
        log(f"{name}: {min(ts) * 1e6:.1f} us (median {np.median(ts) * 1e6:.1f}), orth {orth:.2e}")
        if name == "cholqr2":
            # the same call captured in a HIP graph: one graph launch per factorisation
            g = plan.capture(Z, Q, R)
            g.replay()
            torch.cuda.synchronize()
            ts = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                g.replay()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            orth, res = oqr.check(A, Z, Q, R)
            out["cholqr2_graph"] = {"us_min": round(min(ts) * 1e6, 1),
                                    "us_median": round(float(np.median(ts)) * 1e6, 1),
                                    "orth_loss_fro": orth, "residual_fro": res, "info": int(plan.info.item())}
            log(f"cholqr2 (graph replay): {min(ts) * 1e6:.1f} us (median {np.median(ts) * 1e6:.1f})")
    # the oracle (CHOL-EQR) on the same problem, repeated for about two seconds
    from threadpoolctl import threadpool_info
    from oracle import reference
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 2.0:
        reference.chol_eqr(a, z)
        reps += 1
    tc = (time.perf_counter() - t0) / reps
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    c2 = out["cholqr2"]
    line = {
        "metric": METRIC, "value": round(flops / (c2["us_median"] * 1e-6) / 1e9, 3), "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(c2["us_median"] / 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dense SPD A m={m} n={n} kappa(A)=1e4 kappa(Z)=1e3 (Haar), every variant FP64",
                   "flops_per_step": flops, "flop_count": "2m^2n+2mn^2 (paper normalisation)"},
        "variants_latency": out,
        "roofline": None,
        "roofline_note": "about 1e7 flops per factorisation: launch- and latency-bound, no roofline fraction",
        "cpu_baseline": {"value": round(flops / tc / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
                         "sample": f"chol_eqr on the whole problem, {reps} repetitions", "us_per_call": round(tc * 1e6, 1)},
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (sharded, each "
              "GPU would hold a row block of Z and Q and the passes would all-reduce the n x n Gram)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1401_5171_amd as oqr
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    oqr.lib()   # fail loudly if the library is missing
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return run_batch(args, torch, oqr)
    if args.workload == "copycal":
        return run_copycal(torch)
    if args.workload == "small500":
        return run_small(args, torch, oqr)
    A, Z, z_host, m, n, desc, flops, dom_kernel, dom_flops = make_inputs(args.workload, torch)
    dense = not hasattr(A, "nx") and not hasattr(A, "host")
    # pass 1 of the mixed schedule: hi/lo bfloat16 operands (two slices, products hi*hi + hi*lo + lo*hi),
    # FP32 accumulation, as the workloads specify; pass 2 FP64
    pass1 = args.pass1 or "bf16x2"
    Q = torch.empty(n, m, dtype=torch.float64, device="cuda").t()
    R = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
    mixed = oqr.Plan("cholqr2", A, n, pass1=pass1, pass2="fp64")
    fp64 = oqr.Plan("cholqr2", A, n, pass1="fp64", pass2="fp64")
    fp64_1 = oqr.Plan("cholqr", A, n, pass1="fp64")

    for _ in range(args.warmup):
        mixed.run(Z, Q, R)
        fp64.run(Z, Q, R)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps of each schedule)")

    res = {}
    for name, plan in (("mixed", mixed), ("fp64", fp64)):
        t, kavg, kcnt = time_steps(plan, Z, Q, R, args.steps, torch, dom_kernel)
        orth_f, resid = oqr.check(A, Z, Q, R)
        res[name] = dict(ms_per_step=t * 1e3, kernel_avg_ms=kavg, kernel_launches=kcnt, orth_fro=orth_f,
                         residual_fro=resid, gflops=flops / t / 1e9, breakdown_ms=breakdown(plan, Z, Q, R, torch))
        log(f"{name}: {t * 1e3:.3f} ms/step, {flops / t / 1e9:.1f} GFLOP/s, orth_F={orth_f:.2e} res={resid:.2e}")
    # single FP64 pass (the paper's CHOLQR) for context
    t1, _, _ = time_steps(fp64_1, Z, Q, R, args.steps, torch, dom_kernel)
    orth1, _ = oqr.check(A, Z, Q, R)

    mx = res["mixed"]
    # the stencil's FP64 Gram is the fused A Z + Z^T W kernel in both passes of the FP64 schedule only
    use_fp64 = not mx["kernel_launches"] or (not dense and dom_kernel == "gram")
    kernel_ms = res["fp64"]["kernel_avg_ms"] if use_fp64 else mx["kernel_avg_ms"]
    achieved = dom_flops / (kernel_ms * 1e-3)
    peak = PEAK["fp64"]
    label = (" (FP64, upper block triangle of A with its diagonal blocks, pass 2)" if dense else
             " (FP64 substitution)" if dom_kernel == "trsm" else
             " (fused stencil A Z and Gram Z^T A Z, FP64 schedule, with its partial reduction)")
    roof = {"bound": "mfma", "kernel": dom_kernel + label,
            "achieved": round(achieved / 1e12, 3), "peak": round(peak / 1e12, 1), "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": TRAFFIC.get((args.workload, dom_kernel)),
            "traffic_unit": "L2-miss bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated); "
                            "includes reads the MALL serves, so an upper bound on HBM bytes",
            "per_launch_flops": dom_flops, "avg_launch_ms": round(kernel_ms, 4)}
    line = {
        "metric": METRIC,
        "value": round(mx["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{pass1}+f64",
        "data": "synthetic",
        "config": dict(desc, schedule=f"CholQR2-A pass1={pass1} pass2=fp64", flops_per_step=flops,
                       flop_count="2m^2n+2mn^2 (paper normalisation)" if dense else "2mn^2"),
        "orth_loss_fro": mx["orth_fro"],
        "residual_fro": mx["residual_fro"],
        "fp64_cholqr2": {"value": round(res["fp64"]["gflops"], 2), "ms_per_step": round(res["fp64"]["ms_per_step"], 4),
                         "orth_loss_fro": res["fp64"]["orth_fro"]},
        "fp64_cholqr_single_pass": {"value": round(flops / t1 / 1e9, 2), "ms_per_step": round(t1 * 1e3, 4),
                                    "orth_loss_fro": orth1},
        "speedup_vs_fp64_cholqr2": round(res["fp64"]["ms_per_step"] / mx["ms_per_step"], 3),
        "breakdown_ms": {"mixed": mx["breakdown_ms"], "fp64": res["fp64"]["breakdown_ms"]},
        "roofline": roof,
    }
    kind = "dense" if dense else ("tridiag" if args.workload == "tridiag" else "stencil")
    line["schedule_roofline"] = {
        "mixed": schedule_roofline(kind, m, n, (pass1, "fp64"), mx["ms_per_step"]),
        "fp64": schedule_roofline(kind, m, n, ("fp64", "fp64"), res["fp64"]["ms_per_step"]),
        "definition": "sum over passes of max(unique algorithmic bytes / 8 TB/s, sum of step flops / peak of "
                      "the step's precision); dense A Z and Gram counted as the symmetric schedule executes "
                      "them (upper block triangle of A, about m^2 n + 2 m n^2 per pass)",
    }
    if args.workload == "tridiag":
        line["variants"] = time_variants(A, Z, m, n, flops, torch)
    if args.cpu_sample:
        log("timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(A, z_host, n, min(args.cpu_sample, m), torch)
    else:
        line["cpu_baseline"] = None
    if args.workload == "dense32768" and not args.no_others:
        del A, Z, Q, R, mixed, fp64, fp64_1
        torch.cuda.empty_cache()
        line["other_workloads"] = {"stencil": summary_stencil(args, torch, oqr),
                                   "batch_fp64": summary_batch(args, torch, oqr)}
    print(json.dumps(line), flush=True)


def summary_stencil(args, torch, oqr):
    """The stencil workload (7-point Laplacian + 1e-3 I on 128 x 128 x 64, n = 128, column-scaled Z
    with kappa 1e4): both CholQR2-A schedules timed as the default workload's, with their schedule
    rooflines and the fused FP64 Gram's average launch."""
    A, Z, _, m, n, desc, flops, _, dom_flops = make_inputs("stencil", torch)
    Q = torch.empty(n, m, dtype=torch.float64, device="cuda").t()
    R = torch.empty(n, n, dtype=torch.float64, device="cuda").t()
    out = {"workload": desc["workload"]}
    for name, p1 in (("mixed", "bf16x2"), ("fp64", "fp64")):
        plan = oqr.Plan("cholqr2", A, n, pass1=p1, pass2="fp64")
        for _ in range(args.warmup):
            plan.run(Z, Q, R)
        t, kavg, _ = time_steps(plan, Z, Q, R, args.steps, torch, "gram")
        orth_f, _ = oqr.check(A, Z, Q, R)
        out[name] = {"ms_per_step": round(t * 1e3, 4), "value": round(flops / t / 1e9, 2),
                     "orth_loss_fro": orth_f, "gram_avg_launch_ms": round(kavg, 4),
                     "breakdown_ms": breakdown(plan, Z, Q, R, torch),
                     "schedule_roofline": schedule_roofline("stencil", m, n, (p1, "fp64"), t * 1e3)}
        log(f"stencil {name}: {t * 1e3:.3f} ms/step, orth_F={orth_f:.2e}")
    out["unit"] = "GFLOP/s (2mn^2 per factorisation)"
    return out


def summary_batch(args, torch, oqr):
    """The batch workload (4096 instances, FP64 storage) in one persistent launch: time per launch with
    the autotuned configuration and the launch's fraction of the HBM and FP64-MFMA peaks (bytes and
    flops the symmetric schedule executes)."""
    import argparse as _ap
    import contextlib
    import io
    sub = _ap.Namespace(**vars(args))
    sub.batch_count, sub.batch_dtype, sub.retune, sub.cpu_sample = 4096, "f64", False, 0
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        run_batch(sub, torch, oqr, per_instance=False)
    rec = json.loads(buf.getvalue().strip().splitlines()[-1])
    torch.cuda.empty_cache()
    keep = ("value", "ms_per_step", "orth_loss_fro_max_sampled", "residual_fro_max_sampled", "tuning", "roofline")
    return dict({"workload": rec["config"]["workload"]}, **{k: rec[k] for k in keep})


if __name__ == "__main__":
    main()
