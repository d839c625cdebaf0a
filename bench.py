#!/usr/bin/env python
"""Benchmark of the DtN / Jacobian hot path on one MI355X.

Metric: Jacobian column-steps/s = M * nsteps / wall time of one shoot_eval (residual,
Jacobian and dr/dT) on the precision-form workload: h = 0.5, tau = 0.02, N = 1024,
M = 128 Jacobian columns, 600 DOP853 steps to T/4 (7200 dense DtN evaluations with
one LU each).  One benchmark "step" is one full shoot_eval.  Inputs are the seeded
synthetic surface of the workload, resident in HBM before timing starts.  `value` is
the FP64 form; the FP32-LU + FP64-refinement form is timed the same way and reported
in "mixed".

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 (vector and MFMA)
FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 MFMA
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E

# HBM bytes of the block LU at N = 1024, FP64, LU groups of two stages, from the
# FETCH_SIZE and WRITE_SIZE counter passes in profiles/block_lu_c3_hbm_counters.md,
# calibrated with a plain 256 MiB copy: per k_blu_step launch (averaged over the 15
# steps of a sequence) and per launch sequence (init, 15 steps, final, explicit
# inverse).  Valid only for the kernel source they were measured on: reported as null
# once the kernels header changes.
BLU_STEP_TRAFFIC_BYTES = 26.57e6
LU_SEQ_TRAFFIC_BYTES = 483.3e6
LU_TRAFFIC_SOURCE_SHA256 = "020bbe7fa62336249d1675eb422202b8b7a861eb98a99b27e83be4f92382c65f"
LU_TRAFFIC_GROUP = 2


def lu_traffic_valid():
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1210_5672_amd", "csrc", "ww_kernels.hpp")
    try:
        with open(path, "rb") as fh:
            return hashlib.sha256(fh.read()).hexdigest() == LU_TRAFFIC_SOURCE_SHA256
    except OSError:
        return False


def blu_step_flops(N: int, b: int = 64) -> float:
    """Algorithmic LU flops of the k_blu_step launches of one factorisation: step k
    forms the m = nb - k - 1 left factors L_ik = A_ik D_k (2 b^3 each) and updates the
    m^2 trailing tiles (2 b^3 each), i.e. 2 b^3 (m^2 + m); summed over the steps this is
    2/3 N^3 up to the diagonal-block inversions.  The accumulation of the block-triangular
    inverses that the same launches carry is not counted."""
    nb = N // b
    return sum(2.0 * b ** 3 * (m * m + m) for m in range(1, nb))


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())


def cpu_baseline(w, nsteps_sample: int):
    """The CPU oracle on a bounded prefix of the same workload (same dt), on the
    host's cores: column-steps/s = M * steps / wall time."""
    from oracle import ww_oracle as O
    t0 = time.perf_counter()
    O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params,
                 w.T * nsteps_sample / w.nsteps, nsteps_sample)
    t = time.perf_counter() - t0
    return {"value": w.M * nsteps_sample / t, "unit": "column-steps/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"first {nsteps_sample} of {w.nsteps} RK steps of the same workload, same dt "
                      f"({nsteps_sample * 12 + 1} dense DtN evaluations with J, {t:.1f} s)"}


def run(w, nsteps, T, mixed, steps, warmup, profile, tuned=True):
    """Time `steps` evaluations of shoot_eval after `warmup` ones, without the profiling
    stamps; then, when asked, one more evaluation with the in-graph timestamp nodes for
    the phase durations (which the stamps themselves lengthen a little).  With `tuned`,
    the context takes the autotuner's cached choices for this workload, if any."""
    import torch
    from paper_1210_5672_amd import autotune, ww
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1, mixed=mixed)
    from_cache = bool(autotune.apply(ctx, w.N, w.M)) if tuned else False
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    params = ww.to_dev(w.params)
    tag = "mixed" if mixed else "fp64"
    first_ms = None
    for i in range(warmup):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ctx.shoot_eval(params, T, nsteps)
        if i == 0:   # the first call captures and instantiates the step graphs
            first_ms = 1e3 * (time.perf_counter() - ta)
        print(f"# {tag} warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    each = []
    for i in range(steps):
        ta = time.perf_counter()
        res = ctx.shoot_eval(params, T, nsteps)   # synchronises (status check)
        each.append(1e3 * (time.perf_counter() - ta))
        print(f"# {tag} step {i + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    phases = None
    if profile:
        ctx.profile(True, kernel_events=True)
        ctx.shoot_eval(params, T, nsteps)   # captures the graphs with the stamp nodes
        ctx.profile(True, kernel_events=True)   # clear the sums
        ta = time.perf_counter()
        ctx.shoot_eval(params, T, nsteps)
        prof_ms = 1e3 * (time.perf_counter() - ta)
        lu_ms, lu_n = ctx.profile_stats(0)
        try:   # HIP events around every k_blu_step launched outside a graph
            step_ms, step_n = ctx.profile_stats(4)
        except ww.WWError:
            step_ms, step_n = None, 0
        phases = {"block_lu_ms": lu_ms, "base_chain_ms": ctx.profile_read(1),
                  "column_chain_ms": ctx.profile_read(2),
                  "host_enqueue_ms_per_step": ctx.profile_read(3),
                  # stages factored per LU launch sequence (the lagged march factors
                  # consecutive stages together)
                  "lu_stages_per_sequence": nsteps * 12 / lu_n,
                  "blu_step_ms": step_ms, "blu_step_launches": step_n,
                  "profiled_eval_ms": prof_ms}
        print(f"# {tag} profiled evaluation done", file=sys.stderr, flush=True)
    timing = {"median_ms": statistics.median(each), "min_ms": min(each), "max_ms": max(each),
              "first_call_ms": first_ms, "tuning": ctx.tuning(), "tuning_from_cache": from_cache}
    return t, res, phases, timing


def oracle_fixture(name):
    """Stored FP64 oracle results of a workload (tests/golden/<name>_oracle.npz, written by
    tests/golden/make_oracle_fixtures.py from the CPU oracle), or None."""
    import numpy as np
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", f"{name}_oracle.npz")
    if not os.path.exists(p):
        return None
    fx = np.load(p)
    return fx if "J" in fx.files else None


def err_vs_oracle(res, fx):
    """Relative errors against the stored oracle: r, J (Frobenius, and the largest
    column error on the column's own norm), dr/dT, f; with the oracle's FP64 rounding
    floor (largest spread of its alternate roundings) beside each."""
    import numpy as np
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    J, Jo = res["J"].cpu().numpy(), fx["J"]
    r, d = res["r"].cpu().numpy(), res["drdT"].cpu().numpy()
    out = {"r": rel(r, fx["r"]), "J": rel(J, Jo), "drdT": rel(d, fx["drdT"]),
           "f": abs(res["f"] - float(fx["f"])) / abs(float(fx["f"]))}
    if "alt_r" in fx.files:
        out["floor"] = {"r": float(np.max(fx["alt_r"])), "J": float(np.max(fx["alt_Jfro"])),
                        "drdT": float(np.max(fx["alt_drdT"])), "f": float(np.max(fx["alt_f"]))}
    return out


def run_adjoint(reps: int = 2):
    """Differentiation form (the C4 workload: infinite depth, N = 512, 256 parameters,
    800 steps, checkpoints every 16): time of the gradient by the discrete adjoint
    (shoot_adjoint: forward march with checkpoints, then the reverse sweep with the
    segments recomputed) against the time of the forward f alone (shoot_eval without
    the Jacobian), the ratio the paper discusses for the adjoint method (Sec. 3.2)."""
    import torch
    from paper_1210_5672_amd import workloads as W
    from paper_1210_5672_amd import ww
    w = W.c4()
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1)
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params)
    ctx.shoot_eval(p, w.T, w.nsteps, jacobian=False)
    ctx.shoot_adjoint(p, w.T, w.nsteps, w.ckpt_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.shoot_eval(p, w.T, w.nsteps, jacobian=False)
    tf = (time.perf_counter() - t0) / reps
    print("# adjoint: forward f timed", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.shoot_adjoint(p, w.T, w.nsteps, w.ckpt_every)
    tg = (time.perf_counter() - t0) / reps
    print("# adjoint: gradient timed", file=sys.stderr, flush=True)
    return {"workload": f"C4: N={w.N}, M={w.M}, nsteps={w.nsteps}, checkpoints every {w.ckpt_every}",
            "f_ms": 1e3 * tf, "grad_ms": 1e3 * tg, "grad_over_f": tg / tf}


def run_mesh(reps: int = 2, tuned: bool = True):
    """Time segments on non-uniform meshes (the C6 workload: two segments, N 768 then
    1024 with the mesh refined near x = pi, 24 + 144 steps, 200 parameters):
    shoot_eval_segments, column-steps/s = M x (total steps) / wall time, with the error
    against the stored oracle run when present."""
    import torch
    from paper_1210_5672_amd import autotune, workloads as W
    from paper_1210_5672_amd import ww
    w = W.c6()
    nmax = max(q["N"] for q in w.segments)
    ctx = ww.Context(n_max=nmax, r_max=w.M + 1)
    from_cache = bool(autotune.apply(ctx, nmax, w.M, segments=True)) if tuned else False
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params)
    res = ctx.shoot_eval_segments(p, w.T, w.segments)   # captures the step graphs
    torch.cuda.synchronize()
    each = []
    for _ in range(reps):
        t0 = time.perf_counter()
        res = ctx.shoot_eval_segments(p, w.T, w.segments)
        each.append(time.perf_counter() - t0)
    print("# mesh segments timed", file=sys.stderr, flush=True)
    steps = sum(q["nsteps"] for q in w.segments)
    t = statistics.median(each)
    out = {"workload": w.description, "value": w.M * steps / t, "unit": "column-steps/s", "ms": 1e3 * t,
           "fallbacks": ctx.fallbacks(), "tuning": ctx.tuning(), "tuning_from_cache": from_cache}
    fx = oracle_fixture("c6")
    if fx is not None:
        out["err_vs_oracle"] = err_vs_oracle(res, fx)
    ctx.close()
    return out


def run_sdc(reps: int = 2, sdc_steps: int = 12, low_modes: int = 32, tuned: bool = True):
    """SDC15 (shoot_eval_sdc) on C4 (N 512, infinite depth, no tension, 256 parameters)
    to T/4 in `sdc_steps` steps (113 right-hand-side evaluations each) against the DOP853
    march of the same workload (800 steps of 12 evaluations), each timed with the
    Jacobian and without (f-only), and the two marches' differences: r, dr/dT and the
    Jacobian columns of modes 1..low_modes agree to about 1e-12 (the base march and the
    low modes are resolved by both step sizes); the higher modes carry SDC's larger
    time-discretisation error at this step (omega dt up to 2 at mode 256) and are
    damped by the per-step filter 12 times instead of 800.  With the SDC march's error
    against the stored SDC oracle run when present."""
    import torch
    from paper_1210_5672_amd import autotune
    from paper_1210_5672_amd import workloads as W
    from paper_1210_5672_amd import ww
    w = W.c4()
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1)
    from_cache = bool(autotune.apply(ctx, w.N, w.M)) if tuned else False   # both marches use the choices
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params)

    def timed(fn, n):
        fn()   # first call: work arrays, factor sets, step graphs
        torch.cuda.synchronize()
        each = []
        for _ in range(n):
            t0 = time.perf_counter()
            res = fn()
            each.append(time.perf_counter() - t0)
        return res, statistics.median(each)

    sdc, t_sdc = timed(lambda: ctx.shoot_eval_sdc(p, w.T, sdc_steps), reps)
    fb = ctx.fallbacks()
    sdc_f, t_sdc_f = timed(lambda: ctx.shoot_eval_sdc(p, w.T, sdc_steps, jacobian=False), reps)
    # f-only on GMRES base solves (no LU): a WW_GMRES context
    cg = ww.Context(n_max=w.N, r_max=w.M + 1, gmres=True)
    if tuned:
        autotune.apply(cg, w.N, w.M)
    cg.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    sdc_g, t_sdc_g = timed(lambda: cg.shoot_eval_sdc(p, w.T, sdc_steps, jacobian=False), reps)
    fb_g = cg.fallbacks()
    cg.close()
    rk, t_rk = timed(lambda: ctx.shoot_eval(p, w.T, w.nsteps), 1)
    rk_f, t_rk_f = timed(lambda: ctx.shoot_eval(p, w.T, w.nsteps, jacobian=False), 1)
    print("# SDC15 march timed", file=sys.stderr, flush=True)
    ev = 113 * sdc_steps
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    L = low_modes
    out = {"workload": f"C4: N={w.N}, h=inf, M={w.M}, to T/4 in {sdc_steps} SDC15 steps ({ev} evaluations) "
                       f"vs {w.nsteps} DOP853 steps ({12 * w.nsteps})",
           "with_jacobian": {"sdc_ms": 1e3 * t_sdc, "dop853_ms": 1e3 * t_rk, "speedup": t_rk / t_sdc,
                             "us_per_evaluation": 1e6 * t_sdc / ev},
           "f_only": {"sdc_ms": 1e3 * t_sdc_f, "dop853_ms": 1e3 * t_rk_f, "speedup": t_rk_f / t_sdc_f,
                      "us_per_evaluation": 1e6 * t_sdc_f / ev,
                      "gmres": {"sdc_ms": 1e3 * t_sdc_g, "us_per_evaluation": 1e6 * t_sdc_g / ev, "fallbacks": fb_g,
                                "r_vs_lu": rel(sdc_g["r"], sdc_f["r"])}},
           "fallbacks": fb, "tuning_from_cache": from_cache,
           "sdc_vs_dop853": {"r": rel(sdc["r"], rk["r"]), "drdT": rel(sdc["drdT"], rk["drdT"]),
                             "r_f_only": rel(sdc_f["r"], rk_f["r"]),
                             f"J_modes_1_{L}": rel(sdc["J"][:, :L], rk["J"][:, :L]),
                             "J_all_modes": rel(sdc["J"], rk["J"])}}
    fx = oracle_fixture("c4s")
    if fx is not None:
        out["err_vs_oracle"] = err_vs_oracle(sdc, fx)
    ctx.close()
    return out


def run_sdc_dd(steps=(12, 24, 48)):
    """The base march in double-double with SDC15 (shoot_eval_sdc_dd) on C4's grid and
    initial state (N 512, infinite depth, no tension) to T/4, at each step count in
    `steps`: wall time, time per right-hand-side evaluation, the differences between
    consecutive step counts (SDC15's convergence, followed below the FP64 rounding), and
    the difference from the FP64 SDC march at the first step count."""
    import numpy as np
    import torch
    from paper_1210_5672_amd import workloads as W
    from paper_1210_5672_amd import ww
    w = W.c4()
    N = w.N
    q0 = ww.to_dev(w.q_fixed + w.basis @ w.params)
    ctx = ww.Context(n_max=N, r_max=2)
    ctx.shoot_eval_sdc_dd(N, w.h, w.tau, w.g, q0, None, w.T / 12, 1)   # work arrays, tables
    torch.cuda.synchronize()
    runs = []
    for ns in steps:
        t0 = time.perf_counter()
        o = ctx.shoot_eval_sdc_dd(N, w.h, w.tau, w.g, q0, None, w.T, ns)
        t = time.perf_counter() - t0
        runs.append((ns, t, o["r"][0].cpu().numpy(), o["r"][1].cpu().numpy(), o["f"]))
    # the same march with FP32 factors on MFMA for the corrections (a mixed context)
    cm = ww.Context(n_max=N, r_max=2, mixed=True)
    cm.shoot_eval_sdc_dd(N, w.h, w.tau, w.g, q0, None, w.T / 12, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om = cm.shoot_eval_sdc_dd(N, w.h, w.tau, w.g, q0, None, w.T, steps[0])
    t_mixed = time.perf_counter() - t0
    cm.close()
    mixed_run = (steps[0], t_mixed, om["r"][0].cpu().numpy(), om["r"][1].cpu().numpy(), om["f"])
    print("# double-double SDC15 march timed", file=sys.stderr, flush=True)
    ctx.shoot_setup(N, w.h, w.tau, w.g, ww.to_dev(np.zeros((2 * N, 1))), q0)
    r64 = ctx.shoot_eval_sdc(ww.to_dev(np.zeros(1)), w.T, steps[0], jacobian=False)["r"].cpu().numpy()
    ctx.close()
    scale = np.abs(runs[0][2]).max()
    # differences of double-double values: the hi parts nearly cancel (exactly) plus the
    # lo parts; the low-mode part (k <= 32) of a difference by an FFT of the difference
    # itself (its own rounding is relative to the small difference)
    d = lambda a, b: (a[2] - b[2]) + (a[3] - b[3])
    diff = lambda a, b: float(np.abs(d(a, b)).max() / scale)
    low = lambda a, b: float(np.abs(np.fft.rfft(d(a, b))[:33]).max() / np.abs(np.fft.rfft(runs[0][2])).max())
    out = {"workload": f"C4 grid and initial state, base march to T/4 in double-double, N={N}",
           "marches": [{"steps": ns, "ms": 1e3 * t, "us_per_evaluation": 1e6 * t / (113 * ns + 1), "f": list(f)}
                       for ns, t, _, _, f in runs],
           "r_change_when_halving_dt": [diff(runs[i], runs[i + 1]) for i in range(len(runs) - 1)],
           "r_modes_0_32_change_when_halving_dt": [low(runs[i], runs[i + 1]) for i in range(len(runs) - 1)],
           "f_change_when_halving_dt": [abs((runs[i][4][0] - runs[i + 1][4][0]) + (runs[i][4][1] - runs[i + 1][4][1]))
                                        / runs[0][4][0] for i in range(len(runs) - 1)],
           "r_vs_fp64_sdc": float(np.abs(runs[0][2] + runs[0][3] - r64).max() / scale),
           "fp32_factors": {"steps": steps[0], "ms": 1e3 * t_mixed,
                            "us_per_evaluation": 1e6 * t_mixed / (113 * steps[0] + 1),
                            "r_vs_fp64_factors": diff(mixed_run, runs[0])}}
    return out


def run_dd(reps: int = 3, N: int = 1024, R: int = 129):
    """Double-double DtN (dtn_setup_dd, dtn_solve_multi_dd) on the C3 surface with R
    right-hand sides: set-up time (double-double assembly and FFTs, FP64 LU) and solve
    time (three refinement sweeps and the final residual, each a double-double product
    of A with the R columns, the FFTs and the Gm product).  The products' rate is given
    in FP64 operations at 29 per double-double multiply-add (two-product 2, cross terms
    4, renormalisation 3, accurate addition 20), against the FP64 vector peak."""
    import numpy as np
    import torch
    from paper_1210_5672_amd import workloads as W
    from paper_1210_5672_amd import ww
    w = W.c3()
    eta, _ = W.initial_state(w)
    rhs = np.ascontiguousarray(W.random_rhs(N, R, seed=1210))
    ctx = ww.Context(n_max=N, r_max=R)
    s_hi, r_hi = ww.to_dev(eta), ww.to_dev(rhs)
    ctx.dtn_setup_dd(s_hi, None, w.h)
    ctx.dtn_solve_multi_dd(r_hi, None)
    torch.cuda.synchronize()
    ts, tv = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.dtn_setup_dd(s_hi, None, w.h)
        t1 = time.perf_counter()
        ctx.dtn_solve_multi_dd(r_hi, None)
        t2 = time.perf_counter()
        ts.append(t1 - t0)
        tv.append(t2 - t1)
    print("# double-double DtN timed", file=sys.stderr, flush=True)
    solve = statistics.median(tv)
    madds = 5.0 * N * N * R   # four residual products and the Gm product
    ctx.close()
    return {"workload": f"C3 surface, N={N}, {R} right-hand sides", "setup_ms": 1e3 * statistics.median(ts),
            "solve_ms": 1e3 * solve, "products_fp64_tflops_equiv": 29.0 * madds / solve / 1e12,
            "fp64_vector_peak_tflops": FP64_PEAK_TFLOPS}


def stage_roofline(N, M, nst, stage_ms):
    """Whole-stage roofline: the algorithmic work of one stage at the FP64 MFMA peak and
    the HBM bandwidth, summed phase by phase (each phase at its own bound), against the
    measured stage time.  Flops: LU 2/3 N^3, solve 2 N^2 R, Gm product 2 N^2 R (R = M + 1).
    Bytes: assembly writes of A and Gm (2 N^2 x 8) and the stage combination (on average
    (nst - 1)/2 earlier stage slopes and the state read, the stage state written: 2 N R x 8
    each)."""
    R = M + 1
    t_flop = ((2.0 / 3.0) * N ** 3 + 4.0 * N * N * R) / (FP64_PEAK_TFLOPS * 1e12)
    bytes_ = 2.0 * N * N * 8 + ((nst - 1) / 2.0 + 2.0) * 2.0 * N * R * 8
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
    t_roof = t_flop + t_hbm
    return {"t_roof_us": 1e6 * t_roof, "t_meas_us": 1e3 * stage_ms, "frac": t_roof / (stage_ms * 1e-3)}


def run_batch(window: int = 64, reps: int = 1, tuned: bool = True):
    """Batched form: the 32 continuation instances of uneven N, depth, tension, M (each
    its own context and stream), every instance marched over a fixed window of
    `window` steps at its own dt, all issued together by shoot_eval_batch.
    Column-steps/s = sum_i M_i * window / wall time."""
    import torch
    from paper_1210_5672_amd import autotune
    from paper_1210_5672_amd import workloads as W
    from paper_1210_5672_amd import ww
    ws = W.c5()
    cached = autotune.lookup(max(w.N for w in ws), max(w.M for w in ws), False, batch=True) if tuned else None
    ctxs, params, Ts = [], [], []
    for w in ws:
        c = ww.Context(n_max=w.N, r_max=w.M + 1, stream=torch.cuda.Stream())
        if cached:
            c.set_tuning(**cached)
        c.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        ctxs.append(c)
        params.append(ww.to_dev(w.params))
        Ts.append(w.T * window / w.nsteps)      # same dt as the instance's full march
    steps = [window] * len(ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ww.shoot_eval_batch(ctxs, params, Ts, steps)     # first call: graph capture included
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    print("# batch warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ww.shoot_eval_batch(ctxs, params, Ts, steps)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    cols = sum(w.M for w in ws) * window
    return {"workload": f"{len(ws)} continuation instances (N 256..2048, M 32..256), {window}-step window each",
            "value": cols / t, "unit": "column-steps/s", "ms": 1e3 * t,
            "first_call_ms": 1e3 * t_first, "instances": len(ws), "tuning": ctxs[0].tuning(),
            "tuning_from_cache": bool(cached),
            "N": [w.N for w in ws], "M": [w.M for w in ws]}


def run_f_only(w, nsteps, T):
    """f-only fast path: one march of the precision-form workload without Jacobian
    columns (r, dr/dT, f), with LU base solves and with GMRES base solves (WW_GMRES).
    Returns the times of the second call of each (the first captures the step graph)."""
    import numpy as np
    import torch
    from paper_1210_5672_amd import ww
    out = {"workload": f"base-only march, N={w.N}, nsteps={nsteps} ({12 * nsteps} DtN solves)"}
    rs = {}
    for name, gm in (("lu", False), ("gmres", True)):
        ctx = ww.Context(n_max=w.N, r_max=w.M + 1, gmres=gm)
        ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        params = ww.to_dev(w.params)
        ctx.shoot_eval(params, T, nsteps, jacobian=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.shoot_eval(params, T, nsteps, jacobian=False)
        dt = time.perf_counter() - t0
        rs[name] = res["r"].cpu().numpy()
        out[name] = {"ms": 1e3 * dt, "us_per_stage": 1e6 * dt / (12 * nsteps), "fallbacks": ctx.fallbacks()}
        print(f"# f-only {name} done", file=sys.stderr, flush=True)
    out["r_rel_diff"] = float(np.abs(rs["gmres"] - rs["lu"]).max() / np.abs(rs["lu"]).max())
    out["speedup"] = out["lu"]["ms"] / out["gmres"]["ms"]
    return out


def _standing_wave(N, a1, nmodes):
    """Standing-wave shooting problem (eta even / phi odd modes, basis 2 cos(k alpha),
    c_1 = phi^_1 = a1 fixed; unknowns T and c_2..c_nmodes; infinite depth, g = 1)."""
    import numpy as np
    a = 2 * np.pi * np.arange(N) / N
    ks = list(range(2, nmodes + 1))
    basis = np.zeros((2 * N, len(ks)))
    for j, k in enumerate(ks):
        basis[(0 if k % 2 == 0 else N):(N if k % 2 == 0 else 2 * N), j] = 2 * np.cos(k * a)
    qf = np.concatenate([np.zeros(N), 2 * a1 * np.cos(a)])
    return basis, qf, np.concatenate([[2 * np.pi], np.zeros(len(ks))])


def run_lm(with_oracle: bool):
    """Levenberg-Marquardt row: the thin SVD of a Jacobian of the precision-form shape
    (1024 x 129), a standing-wave solve at N = 256 (nsteps 128, 31 unknown modes and T),
    and the GPU driver against the oracle driver on a small standing wave (N = 64)."""
    import math
    import numpy as np
    import torch
    from paper_1210_5672_amd import ww
    rng = np.random.default_rng(1210)
    A = ww.to_dev(rng.standard_normal((1024, 129)))
    cs = ww.Context(n_max=1024, r_max=129)
    cs.thin_svd(A)
    t0 = time.perf_counter()
    for _ in range(3):
        cs.thin_svd(A)
    svd_ms = 1e3 * (time.perf_counter() - t0) / 3
    out = {"svd_1024x129_ms": svd_ms}
    solves = {}
    for (N, nsteps, nmodes) in [(256, 128, 32), (64, 32, 10)]:
        basis, qf, c0 = _standing_wave(N, 0.05, nmodes)
        ctx = ww.Context(n_max=N, r_max=nmodes)
        ctx.shoot_setup(N, math.inf, 0.0, 1.0, ww.to_dev(basis), ww.to_dev(qf))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.levmar(c0, nsteps, opts={"delta0": 0.1, "max_evals": 80})
        dt = time.perf_counter() - t0
        solves[N] = {"N": N, "nsteps": nsteps, "unknowns": nmodes, "ms": 1e3 * dt, "f": res["f"],
                     "evals_r": res["evals_r"], "evals_J": res["evals_J"], "reason": res["reason"],
                     "T": float(res["c"][0]), "last_fallbacks": ctx.fallbacks()}
        print(f"# lm N={N} done", file=sys.stderr, flush=True)
    out["standing_wave_n256"] = solves[256]
    out["standing_wave_n64"] = solves[64]
    # BFGS with the adjoint gradient (Sec. 3.2) on a small standing wave
    basis, qf, c0 = _standing_wave(32, 0.05, 10)
    ctx = ww.Context(n_max=32, r_max=10)
    ctx.shoot_setup(32, math.inf, 0.0, 1.0, ww.to_dev(basis), ww.to_dev(qf))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bres = ctx.bfgs(c0, 12, opts={"delta0": 0.1, "max_iter": 80, "ckpt_every": 4})
    out["bfgs_n32"] = {"N": 32, "nsteps": 12, "unknowns": 10, "ms": 1e3 * (time.perf_counter() - t0), "f": bres["f"],
                       "iters": bres["iters"], "evals": bres["evals"], "reason": bres["reason"]}
    if with_oracle:
        from oracle import lm_oracle as L
        from oracle import ww_oracle as O
        N, nsteps, nmodes = 64, 32, 10
        basis, qf, c0 = _standing_wave(N, 0.05, nmodes)

        def jac(c):
            o = O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=True)
            return o["r"], np.concatenate([o["drdT"][:, None], o["J"]], axis=1)

        def resid(c):
            return O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=False)["r"]

        t0 = time.perf_counter()
        ref = L.levmar(resid, jac, c0, delta0=0.1, max_evals=80)
        out["oracle_n64"] = {"ms": 1e3 * (time.perf_counter() - t0), "f": ref.f, "evals_r": ref.evals_r,
                             "evals_J": ref.evals_J, "cores": blas_threads(), "kind": "oracle"}
        from oracle import bfgs_oracle as B
        basis, qf, c0 = _standing_wave(32, 0.05, 10)

        def fg(c):
            o = O.shoot_eval(32, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], 12, jacobian=True)
            J = np.concatenate([o["drdT"][:, None], o["J"]], axis=1)
            return 0.5 * float(o["r"] @ o["r"]), J.T @ o["r"]

        t0 = time.perf_counter()
        bref = B.bfgs(fg, c0, delta0=0.1, max_iter=80)
        out["oracle_bfgs_n32"] = {"ms": 1e3 * (time.perf_counter() - t0), "f": bref.f, "evals": bref.evals,
                                  "cores": blas_threads(), "kind": "oracle"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsteps", type=int, default=None,
                    help="RK step count override (profiling runs only; the line names the count)")
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances measurement")
    ap.add_argument("--no-lm", action="store_true", help="skip the Levenberg-Marquardt measurement")
    ap.add_argument("--no-f-only", action="store_true", help="skip the f-only (GMRES) measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-gradient timing (C4)")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the autotuner's cached choices")
    ap.add_argument("--no-mesh", action="store_true", help="skip the segmented non-uniform-mesh march (C6)")
    ap.add_argument("--no-dd", action="store_true", help="skip the double-double DtN timing")
    ap.add_argument("--no-sdc", action="store_true", help="skip the SDC15 march (C4)")
    ap.add_argument("--no-sdc-dd", action="store_true", help="skip the double-double SDC15 base march (C4 grid)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by Jacobian column or by instance; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    from paper_1210_5672_amd import workloads as W

    w = W.c3()
    nsteps = args.nsteps or w.nsteps
    T = w.T if nsteps == w.nsteps else w.T * nsteps / w.nsteps   # same dt for a prefix
    print(f"# workload {w.name}: N={w.N} M={w.M} nsteps={nsteps}", file=sys.stderr, flush=True)
    profile = not args.no_profile
    t, res, phases, timing = run(w, nsteps, T, False, args.steps, args.warmup, profile, not args.no_tuning)
    ms = 1000.0 * t / args.steps
    value = w.M * nsteps * args.steps / t
    n3 = float(w.N) ** 3
    roofline = None
    if phases:
        # dominant kernel: k_blu_step (15 launches per LU sequence; each launch carries
        # the tasks of the G stages of a group).  Achieved = algorithmic LU flops per
        # launch (the sequence's step flops / launches) over the mean launch duration
        # from HIP events on the launching stream.
        G = phases["lu_stages_per_sequence"]
        nb = w.N // 64
        seq_flops = G * blu_step_flops(w.N)
        valid = lu_traffic_valid() and w.N == 1024 and timing["tuning"]["lu_group"] == LU_TRAFFIC_GROUP
        seq = {"kernels": "k_blu_init, 15 x k_blu_step, k_blu_final, k_minv",
               "stages": G, "ms": phases["block_lu_ms"],
               "achieved": G * (2.0 / 3.0) * n3 / (phases["block_lu_ms"] * 1e-3) / 1e12,
               "traffic": LU_SEQ_TRAFFIC_BYTES if valid else None}
        if phases.get("blu_step_launches"):
            step_s = phases["blu_step_ms"] * 1e-3
            ach = seq_flops / (nb - 1) / step_s / 1e12
            roofline = {"bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / FP64_PEAK_TFLOPS, "traffic": BLU_STEP_TRAFFIC_BYTES if valid else None,
                        "kernel": f"k_blu_step<double>, one launch per block step of a group of {G:g} stages",
                        "flops_per_launch": seq_flops / (nb - 1),
                        "launch_us": phases["blu_step_ms"] * 1e3,
                        "launches_timed": phases["blu_step_launches"],
                        "sequence": seq, "phases_ms": phases}
        else:   # every LU replayed from a graph: no per-launch events, sequence figure only
            roofline = {"bound": "mfma", "achieved": seq["achieved"], "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": seq["achieved"] / FP64_PEAK_TFLOPS,
                        "traffic": seq["traffic"], "kernel": "block LU launch sequence",
                        "sequence": seq, "phases_ms": phases}
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "shoot_eval h=0.5 tau=0.02 N=1024 M=128 nsteps=600 (precision form)",
                   "N": w.N, "M": w.M, "nsteps": nsteps, "f": res["f"], "tuning": timing["tuning"]},
        "roofline": roofline,
        "cpu_baseline": None,
        "timing": timing,
        "stage_roofline": stage_roofline(w.N, w.M, 12, timing["median_ms"] / (nsteps * 12)),
    }
    fx = oracle_fixture("c3") if nsteps == w.nsteps else None
    if fx is not None:
        out["err_vs_oracle"] = err_vs_oracle(res, fx)
    if not args.no_mixed:
        import numpy as np
        tm, resm, phm, timm = run(w, nsteps, T, True, args.steps, args.warmup, profile, not args.no_tuning)
        r64, rm = res["r"].cpu().numpy(), resm["r"].cpu().numpy()
        J64, Jm = res["J"].cpu().numpy(), resm["J"].cpu().numpy()
        out["mixed"] = {
            "value": w.M * nsteps * args.steps / tm, "ms_per_step": 1000.0 * tm / args.steps,
            "dtype": "f32-lu+f64-refine", "timing": timm,
            "rel_diff_vs_fp64": {"r": float(np.linalg.norm(rm - r64) / np.linalg.norm(r64)),
                                 "J": float(np.linalg.norm(Jm - J64) / np.linalg.norm(J64))},
        }
        if fx is not None:
            out["mixed"]["err_vs_oracle"] = err_vs_oracle(resm, fx)
        if phm:
            lu_s = phm["block_lu_ms"] * 1e-3
            ach = phm["lu_stages_per_sequence"] * (2.0 / 3.0) * n3 / lu_s / 1e12
            out["mixed"]["roofline"] = {"bound": "mfma", "achieved": ach, "peak": FP32_PEAK_TFLOPS,
                                        "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                                        "phases_ms": phm}
    # single-instance sections first: the batch creates torch's stream pool, and every
    # stream a process holds changes the hardware queues that later streams are given
    if not args.no_lm:
        out["lm"] = run_lm(with_oracle=not args.no_cpu_baseline)
    if not args.no_f_only:
        out["f_only"] = run_f_only(w, nsteps, T)
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint()
    if not args.no_mesh:
        out["mesh"] = run_mesh(tuned=not args.no_tuning)
    if not args.no_dd:
        out["dd"] = run_dd()
    if not args.no_sdc:
        out["sdc"] = run_sdc(tuned=not args.no_tuning)
    if not args.no_sdc_dd:
        out["sdc_dd"] = run_sdc_dd()
    if not args.no_batch:
        out["batch"] = run_batch(tuned=not args.no_tuning)
    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE under a counter run
        # give the scale between the counters and the bytes actually moved
        import torch
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 8
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
