"""Tune the batched CholQR2-A launch and store the table beside the library.

    python -m paper_1401_5171_amd.tune_batch [--count 4096] [--dtype f64|f32|both] [--out PATH]

Builds the synthetic batch (m log-uniform in [256, 4096], n in {8, 16, 32, 64}, kappa(A_i)
log-uniform in [1e2, 1e8], Gaussian Z_i) on the current device, runs `BatchPlan.autotune` (tile
shape per (m bucket, n class), then workgroups per compute unit) and writes the chosen tuning for
each storage type into the JSON table (default: batch_tuning.json in this package, which BatchPlan
reads when no tuning is given).  Needs a HIP device.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def tune(count: int, dtype: str, out: str, reps: int = 3) -> dict:
    import torch

    import paper_1401_5171_amd as oqr
    import workloads as W
    dev = torch.device("cuda", 0)
    dt = torch.float64 if dtype == "f64" else torch.float32
    sizes = W.batch_plan(count)
    t = time.time()
    As, Zs = [], []
    for p in sizes:
        a, z = W.batch_instance_device(p, dev, dt)
        As.append(a)
        Zs.append(z)
    torch.cuda.synchronize()
    print(f"[tune] {dtype}: {count} instances built in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    plan = oqr.BatchPlan(As, Zs, tuning=oqr.default_batch_tuning())
    report = plan.autotune(reps=reps)
    oqr.save_batch_tuning(plan.tuning, dtype, out)
    print(f"[tune] {dtype}: {json.dumps(report)}", file=sys.stderr, flush=True)
    del plan, As, Zs
    torch.cuda.empty_cache()
    return report


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--count", type=int, default=4096)
    p.add_argument("--dtype", default="both", choices=["f64", "f32", "both"])
    p.add_argument("--out", default=os.path.join(HERE, "batch_tuning.json"))
    p.add_argument("--reps", type=int, default=3)
    args = p.parse_args()
    for d in (("f64", "f32") if args.dtype == "both" else (args.dtype,)):
        tune(args.count, d, args.out, args.reps)
    print(open(args.out).read())


if __name__ == "__main__":
    main()
