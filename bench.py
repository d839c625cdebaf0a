#!/usr/bin/env python
"""Benchmark of the DtN / Jacobian hot path on one MI355X.

Metric: Jacobian column-steps/s = M * nsteps / wall time of one shoot_eval (residual,
Jacobian and dr/dT) on the precision-form workload: h = 0.5, tau = 0.02, N = 1024,
M = 128 Jacobian columns, 600 DOP853 steps to T/4 (7200 dense DtN evaluations with
one LU each).  One benchmark "step" is one full shoot_eval.  Inputs are the seeded
synthetic surface of the workload, resident in HBM before timing starts.

Prints one JSON line (see the repository's design notes for the fields).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time


def cpu_baseline(w, nsteps_sample: int):
    """The CPU oracle on a bounded prefix of the same workload (same dt), on the
    host's cores: column-steps/s = M * steps / wall time."""
    import numpy as np  # noqa: F401
    from oracle import ww_oracle as O
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    t0 = time.perf_counter()
    O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params,
                 w.T * nsteps_sample / w.nsteps, nsteps_sample)
    t = time.perf_counter() - t0
    return {"value": w.M * nsteps_sample / t, "unit": "column-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{nsteps_sample} of {w.nsteps} RK steps of the same workload "
                      f"({nsteps_sample * 12 + 1} DtN evaluations, {t:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--nsteps", type=int, default=None,
                    help="override the RK step count (profiling runs only; the metric "
                         "line names the count used)")
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by Jacobian column or by instance; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1210_5672_amd import workloads as W
    from paper_1210_5672_amd import ww

    w = W.c3()
    nsteps = args.nsteps or w.nsteps
    T = w.T if nsteps == w.nsteps else w.T * nsteps / w.nsteps   # same dt for a prefix
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1, mixed=(args.precision == "mixed"))
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    params = ww.to_dev(w.params)
    print(f"# workload {w.name}: N={w.N} M={w.M} nsteps={nsteps} precision={args.precision}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        ctx.shoot_eval(params, T, nsteps)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for i in range(args.steps):
        res = ctx.shoot_eval(params, T, nsteps)
        print(f"# step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms = 1000.0 * t / args.steps
    value = w.M * nsteps * args.steps / t
    out = {
        "metric": "Jacobian column-steps/s at N=1024",
        "value": value,
        "unit": "column-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-lu+f64-refine",
        "data": "synthetic",
        "config": {"workload": "shoot_eval h=0.5 tau=0.02 N=1024 M=128 (precision form)",
                   "N": w.N, "M": w.M, "nsteps": nsteps, "precision": args.precision,
                   "f": res["f"]},
        "roofline": None,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
