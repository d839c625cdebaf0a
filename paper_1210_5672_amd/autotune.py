"""Autotuner of the launch and scheduling choices of a context (ww_tuning).

None of the choices changes what is computed: they decide how the work of a march is
cut into launches and streams (LU group size and streams, the lag of the base solve,
which parts replay from graphs, the strip length of a block-LU step, rows per
workgroup of the base DtN launch, the inner-dimension split and the output-tile rows
of the column products, the assembly strip width, the workgroup cap of the explicit
inverse, an FP32 copy of the lagged inverse for the base solve's products, the
refinement sweeps of a lagged solve).  The tuner times
short marches of a workload, one fresh context per candidate, and improves one choice
at a time (coordinate descent, a few passes); the winner is stored in a JSON cache
keyed by GPU architecture, N, M and precision form, and `apply` hands it to a context.

A candidate whose march falls back (for instance a lag too short for the refinement
sweeps to converge) is discarded: its time is that of another path.

Command line (on the GPU):
    python -m paper_1210_5672_amd.autotune c3 [--mixed] [--steps 6] [--cache PATH]
    python -m paper_1210_5672_amd.autotune c5 --batch        (the batched instances)
    python -m paper_1210_5672_amd.autotune c6                 (time segments, whole march)
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import tempfile
import time

CACHE_ENV = "WW_TUNING_CACHE"
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")

# candidate values of every choice (the defaults of ww_create are among them)
SPACE = {
    "graph_parts": [10, 0, 15, 2],
    "lu_group": [2, 1, 3, 4],
    "lu_streams": [3, 2, 4],
    "lag": [8, 6, 10],
    "lag_sweeps": [2, 3, 4],
    "blu_strip": [4, 2, 3, 6, 8],
    "minv_wgs": [1 << 20, 256, 128],
    "dtn_rows": [8, 4, 16],
    "gemm_split": [4, 2],
    "asm_cw": [16, 32],
    "gemm_rows": [32, 16],
    "lag_fp32": [0, 1],
}
# choices that matter only to the lagged-factor march (a batch runs each instance's
# own step graph)
MARCH_ONLY = ("graph_parts", "lu_group", "lu_streams", "lag", "dtn_rows", "lag_fp32", "lag_sweeps")


def cache_path(path: str | None = None) -> str:
    return path or os.environ.get(CACHE_ENV) or DEFAULT_CACHE


def arch_name() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def key(N: int, M: int, mixed: bool, arch: str | None = None, batch: bool = False, segments: bool = False) -> str:
    sfx = "/batch" if batch else "/segments" if segments else ""
    return f"{arch or arch_name()}/N{N}/M{M}/{'mixed' if mixed else 'fp64'}{sfx}"


def load(path: str | None = None) -> dict:
    p = cache_path(path)
    if not os.path.exists(p):
        return {}
    with open(p) as fh:
        data = json.load(fh)
    if not isinstance(data, dict):
        raise ValueError(f"{p}: not a tuning cache")
    return data


def save(cache: dict, path: str | None = None) -> str:
    """Write the cache atomically (a temporary file in the same folder, then rename)."""
    p = cache_path(path)
    d = os.path.dirname(os.path.abspath(p))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
        fh.write("\n")
    os.replace(tmp, p)
    return p


def lookup(N: int, M: int, mixed: bool, path: str | None = None, arch: str | None = None,
           batch: bool = False, segments: bool = False) -> dict | None:
    entry = load(path).get(key(N, M, mixed, arch, batch, segments))
    return dict(entry["tuning"]) if entry else None


def apply(ctx, N: int, M: int, path: str | None = None, batch: bool = False, segments: bool = False) -> dict | None:
    """Give `ctx` the cached choices for (N, M, its precision form), if any; returns them.
    Segmented marches (shoot_eval_segments) are keyed by their largest N."""
    t = lookup(N, M, ctx.mixed, path, batch=batch, segments=segments)
    if t:
        ctx.set_tuning(**t)
    return t


def candidates(cur: dict, name: str) -> list:
    return [v for v in SPACE[name] if v != cur[name]]


def descend(measure, start: dict, names, passes: int = 2, min_gain: float = 0.01, log=print):
    """Coordinate descent: `measure(choices) -> seconds or None` (None: rejected).
    When the starting choices themselves fall back, their time on the fallback path
    (`measure(choices, allow_fallback=True)`, the path those choices really take) is the
    baseline that a candidate must beat.  Returns (best choices, best time, history)."""
    best = dict(start)
    t_best = measure(best)
    if t_best is None:
        try:
            t_best = measure(best, allow_fallback=True)
        except TypeError:
            t_best = None
        if t_best is None:
            raise RuntimeError("the starting choices fall back")
        log(f"  the starting choices fall back: baseline {t_best * 1e3:.3f} ms on the fallback path")
    hist = [(dict(best), t_best)]
    for _ in range(passes):
        improved = False
        for name in names:
            for v in candidates(best, name):
                trial = dict(best, **{name: v})
                t = measure(trial)
                hist.append((trial, t))
                log(f"  {name}={v}: " + (f"{t * 1e3:.3f} ms" if t is not None else "rejected (fallback)"))
                if t is not None and t < t_best * (1 - min_gain):
                    best, t_best, improved = trial, t, True
        if not improved:
            break
    return best, t_best, hist


def _march_measure(w, mixed: bool, nsteps: int, reps: int):
    import torch
    from . import ww
    T = w.T * nsteps / w.nsteps
    basis, qfix, params = ww.to_dev(w.basis), ww.to_dev(w.q_fixed), ww.to_dev(w.params)
    segs = w.segments
    nmax = max(q["N"] for q in segs) if segs else w.N

    def march(ctx):
        # a segmented workload is timed whole (its segments are short)
        return ctx.shoot_eval_segments(params, w.T, segs) if segs else ctx.shoot_eval(params, T, nsteps)

    def measure(choices, allow_fallback=False):
        ctx = ww.Context(n_max=nmax, r_max=w.M + 1, mixed=mixed)
        try:
            ctx.set_tuning(**choices)
            ctx.shoot_setup(w.N, w.h, w.tau, w.g, basis, qfix)
            march(ctx)                                 # captures the graphs
            if ctx.fallbacks() and not allow_fallback:
                return None
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                march(ctx)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                if ctx.fallbacks() and not allow_fallback:
                    return None
            return statistics.median(ts)
        finally:
            ctx.close()
    return measure


def _batch_measure(ws, mixed: bool, reps: int):
    import torch
    from . import ww
    inputs = [(ww.to_dev(w.basis), ww.to_dev(w.q_fixed), ww.to_dev(w.params)) for w in ws]

    def measure(choices):
        ctxs = []
        try:
            for w, (b, q, _) in zip(ws, inputs):
                c = ww.Context(n_max=w.N, r_max=w.M + 1, mixed=mixed, stream=torch.cuda.Stream())
                c.set_tuning(**choices)
                c.shoot_setup(w.N, w.h, w.tau, w.g, b, q)
                ctxs.append(c)
            args = ([x[2] for x in inputs], [w.T for w in ws], [w.nsteps for w in ws])
            ww.shoot_eval_batch(ctxs, *args)
            torch.cuda.synchronize()
            if any(c.fallbacks() for c in ctxs):
                return None
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ww.shoot_eval_batch(ctxs, *args)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return statistics.median(ts)
        finally:
            for c in ctxs:
                c.close()
    return measure


def tune(w, mixed: bool = False, nsteps: int = 6, reps: int = 2, passes: int = 2, log=print):
    """Tune the lagged-factor march of workload `w` (its first `nsteps` steps)."""
    from . import ww
    probe = ww.Context(n_max=w.N, r_max=w.M + 1, mixed=mixed)
    start = probe.tuning()
    probe.close()
    return descend(_march_measure(w, mixed, nsteps, reps), start, list(SPACE), passes, log=log)


def tune_batch(ws, mixed: bool = False, reps: int = 2, passes: int = 1, log=print):
    """Tune a batch of instances (shoot_eval_batch), one set of choices for all."""
    from . import ww
    probe = ww.Context(n_max=ws[0].N, r_max=ws[0].M + 1, mixed=mixed)
    start = probe.tuning()
    probe.close()
    names = [n for n in SPACE if n not in MARCH_ONLY]
    return descend(_batch_measure(ws, mixed, reps), start, names, passes, log=log)


def store(k: str, best: dict, t: float, note: str, path: str | None = None) -> str:
    cache = load(path)
    cache[k] = {"tuning": best, "seconds": t, "note": note, "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    return save(cache, path)


def main(argv=None):
    from . import workloads as W
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("workload", help="c1..c4, c6 (time segments), or c5 with --batch")
    ap.add_argument("--mixed", action="store_true")
    ap.add_argument("--batch", action="store_true", help="tune the batched instances (c5)")
    ap.add_argument("--steps", type=int, default=6, help="steps of the timed march prefix")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--instances", type=int, default=32, help="batched instances (--batch)")
    ap.add_argument("--cache", default=None)
    a = ap.parse_args(argv)
    if a.batch:
        ws = [w for w in W.c5()[:a.instances]]
        # each instance's own dt, a few steps each
        ws = [W.Workload(w.name, w.N, w.h, w.tau, w.g, w.M, w.T * min(a.steps, w.nsteps) / w.nsteps,
                         min(a.steps, w.nsteps), w.params, w.basis, w.q_fixed) for w in ws]
        print(f"tuning the batch of {len(ws)} instances, {'mixed' if a.mixed else 'fp64'}", flush=True)
        best, t, _ = tune_batch(ws, a.mixed, a.reps, a.passes)
        k = key(max(w.N for w in ws), max(w.M for w in ws), a.mixed, batch=True)
        note = f"{len(ws)} batched instances, {a.steps}-step prefixes"
    else:
        w = W.CONFIGS[a.workload]()
        segs = w.segments
        print(f"tuning {w.name}, {'mixed' if a.mixed else 'fp64'}, "
              f"{'whole segmented march' if segs else f'{a.steps}-step prefix'}", flush=True)
        best, t, _ = tune(w, a.mixed, a.steps, a.reps, a.passes)
        k = key(max(q["N"] for q in segs) if segs else w.N, w.M, a.mixed, segments=bool(segs))
        note = f"{w.name}, " + ("whole segmented march" if segs else f"{a.steps}-step prefix")
    p = store(k, best, t, note, a.cache)
    print(json.dumps({"key": k, "tuning": best, "seconds": t, "cache": p}), flush=True)


if __name__ == "__main__":
    main()
