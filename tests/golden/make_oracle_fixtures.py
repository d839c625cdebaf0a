"""Write full-size reference results of the CPU oracle for the parity tests.

Calls only oracle/ (and the seeded input generators).  Run from the repository root:

    python tests/golden/make_oracle_fixtures.py run NAME ARITH [A:B]
    python tests/golden/make_oracle_fixtures.py combine NAME
    python tests/golden/make_oracle_fixtures.py all [-j JOBS] [NAME ...]

`run` marches workload NAME with one arithmetic of the oracle and writes
tests/golden/raw/NAME_ARITH[_A-B].npz (r, J, drdT, f):
  f64     the FP64 oracle (the reference the GPU path is compared with);
  alt_cs  FP64 with cosh/sinh from the math library instead of from exp(+-y);
  alt_fft FP64 with the Fourier multipliers through the full complex FFT;
  alt_sum FP64 with the summation order of products and of the solve reversed;
  alt_inv FP64 with every dense solve done through the explicit inverse;
  dd      double-double (about 32 digits), for C1 and C2: the FP64 oracle's error
          itself.  A:B runs Jacobian columns A..B-1 only (the initial state is that of
          all parameters; the columns of the variational march are independent), so
          that the double-double C2 march can run in several processes.
`combine` writes tests/golden/NAME_oracle.npz: the f64 results with the full J, the
gradient J^T r and df/dT, and the rounding floor: for each alternate arithmetic the
relative 2-norm differences of r, f, drdT, grad, J (Frobenius) and, per column of J,
the largest absolute difference; where a double-double run exists, the same measures
of the FP64 oracle's error against it (and NAME_dd.npz holds the double-double
results rounded to doubles).
`all` runs every job of the listed workloads (default: all of them) that has no stored
raw result yet, in parallel processes, one thread each, then combines.  The full set takes about two hours on
8 cores (C3: 7200 dense N = 1024 solves per run, four runs).

Workloads: c1, c2, c3, c4; c5_IIxS, the first S steps of batched instance II (the
largest grids); c5_II, batched instance II marched to T/4 (instances whose oracle
run is affordable); c6, the two time segments on non-uniform meshes (the mesh oracle,
oracle/mesh_oracle.py, with the same FP64 alternates); c4s, C4 marched to T/4 with 12
steps of SDC15 (the SDC oracle, oracle/sdc_oracle.py, with the same FP64 alternates);
c6s, the C6 segments marched by 4 + 15 SDC15 steps (the mesh oracle's SDC march).
"""
import os
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
RAW = os.path.join(HERE, "raw")
sys.path.insert(0, ROOT)

from oracle import mesh_oracle as MO              # noqa: E402
from oracle import sdc_oracle as SO               # noqa: E402
from oracle import ww_oracle as O                 # noqa: E402
from paper_1210_5672_amd import workloads as W   # noqa: E402

ALTS = ("alt_cs", "alt_fft", "alt_sum", "alt_inv")

# prefixes of batched continuation instances at the largest sizes: (instance, steps);
# the march uses the instance's own dt (T scaled with the step count)
C5_PREFIX = {"c5_16x3": (16, 3), "c5_02x3": (2, 3)}
# batched instances marched to T/4 in full (N = 256..512, up to 140 steps; radix-3
# N = 384; the shallow h = 0.198 and h = 0.254 instances)
C5_FULL = {"c5_00": 0, "c5_07": 7, "c5_08": 8, "c5_26": 26, "c5_27": 27}

# workloads with a double-double run, and the column split of that run
DD_SPLIT = {"c1": 1, "c2": 4}
# workloads marched with SDC15: (base workload, SDC steps to T/4)
SDC_RUNS = {"c4s": ("c4", 12)}
# segmented workloads marched with SDC15: (base workload, SDC steps of each segment)
SDC_SEG_RUNS = {"c6s": ("c6", (4, 15))}
ALL = ("c1", "c2", "c4", "c3", *C5_FULL, *C5_PREFIX, "c6", *SDC_RUNS, *SDC_SEG_RUNS)


def workload(name):
    if name in C5_PREFIX:
        idx, steps = C5_PREFIX[name]
        w = W.c5()[idx]
        return W.Workload(name, w.N, w.h, w.tau, w.g, w.M, w.T * steps / w.nsteps, steps, w.params, w.basis,
                          w.q_fixed, description=f"first {steps} steps of batched instance {idx}")
    if name in C5_FULL:
        w = W.c5()[C5_FULL[name]]
        return W.Workload(name, w.N, w.h, w.tau, w.g, w.M, w.T, w.nsteps, w.params, w.basis, w.q_fixed,
                          description=f"batched instance {C5_FULL[name]} to T/4")
    if name in SDC_RUNS:
        base, steps = SDC_RUNS[name]
        w = W.CONFIGS[base]()
        return W.Workload(name, w.N, w.h, w.tau, w.g, w.M, w.T, steps, w.params, w.basis, w.q_fixed,
                          description=f"{base} to T/4 with {steps} SDC15 steps")
    if name in SDC_SEG_RUNS:
        base, steps = SDC_SEG_RUNS[name]
        w = W.CONFIGS[base]()
        segs = [dict(q, nsteps=n) for q, n in zip(w.segments, steps)]
        return W.Workload(name, w.N, w.h, w.tau, w.g, w.M, w.T, sum(steps), w.params, w.basis, w.q_fixed,
                          segments=segs, description=f"{base} segments with {steps} SDC15 steps")
    return W.CONFIGS[name]()


def arith(tag):
    if tag == "dd":
        from oracle import dd
        return dd.DDArith()
    return {"f64": O.F64, "alt_cs": O.F64ALT, "alt_fft": O.F64ALT_FFT, "alt_sum": O.F64ALT_SUM,
            "alt_inv": O.F64ALT_INV}[tag]


def _raw_path(name, tag, cols=None):
    sfx = f"_{cols[0]}-{cols[1]}" if cols else ""
    return os.path.join(RAW, f"{name}_{tag}{sfx}.npz")


def run(name, tag, cols=None):
    w = workload(name)
    ar = arith(tag)
    t0 = time.time()
    if name in SDC_RUNS:
        if cols is not None or tag == "dd":
            raise SystemExit("SDC15 runs are FP64 runs of all columns")
        res = SO.shoot_eval_sdc(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps, ar=ar)
    elif w.segments is not None:
        if cols is not None:
            raise SystemExit("column splits are for uniform-mesh workloads")
        res = MO.shoot_eval_segments(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.segments, ar=ar,
                                     scheme="sdc" if name in SDC_SEG_RUNS else "dop853")
    elif cols is None:
        res = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps, ar=ar)
    else:
        # columns a..b-1 only: the initial state of all parameters, formed in the run's
        # arithmetic exactly as the oracle forms it, enters as the fixed part
        a, b = cols
        q0 = ar.asarray(w.q_fixed) + ar.matmul(ar.asarray(w.basis), ar.asarray(w.params))
        res = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis[:, a:b], q0, np.zeros(b - a), w.T, w.nsteps, ar=ar)
    f = lambda x: np.asarray(x.to_float() if hasattr(x, "to_float") else x, dtype=float)
    os.makedirs(RAW, exist_ok=True)
    out = _raw_path(name, tag, cols)
    np.savez_compressed(out + ".tmp.npz", r=f(res["r"]), J=f(res["J"]), drdT=f(res["drdT"]),
                        f=np.array(float(res["f"])), seconds=np.array(time.time() - t0))
    os.replace(out + ".tmp.npz", out)
    print(name, tag, cols, "done in %.0f s" % (time.time() - t0), "->", out, flush=True)


def _splits(name):
    n = DD_SPLIT.get(name, 0)
    if not n:
        return []
    M = workload(name).M
    step = (M + n - 1) // n
    return [(a, min(M, a + step)) for a in range(0, M, step)]


def _load_raw(name, tag):
    if tag == "dd":
        sp = _splits(name)
        paths = [_raw_path(name, "dd", c if len(sp) > 1 else None) for c in sp]
        if not paths or not all(os.path.exists(p) for p in paths):
            return None
        parts = [np.load(p) for p in paths]
        for p in parts[1:]:   # the base march is the same in every part
            assert np.array_equal(p["r"], parts[0]["r"]) and np.array_equal(p["drdT"], parts[0]["drdT"])
        return {"r": parts[0]["r"], "drdT": parts[0]["drdT"], "f": float(parts[0]["f"]),
                "J": np.hstack([p["J"] for p in parts])}
    p = _raw_path(name, tag)
    if not os.path.exists(p):
        return None
    d = np.load(p)
    return {k: (float(d[k]) if k == "f" else d[k]) for k in ("r", "J", "drdT", "f")}


def _diffs(x, ref):
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"r": rel(x["r"], ref["r"]), "f": abs(x["f"] - ref["f"]) / abs(ref["f"]),
            "drdT": rel(x["drdT"], ref["drdT"]), "grad": rel(x["J"].T @ x["r"], ref["J"].T @ ref["r"]),
            "Jfro": rel(x["J"], ref["J"]), "Jcol": np.abs(x["J"] - ref["J"]).max(axis=0)}


def combine(name):
    w = workload(name)
    ref = _load_raw(name, "f64")
    if ref is None:
        raise SystemExit(f"{name}: no f64 run")
    grad = ref["J"].T @ ref["r"]
    dfdT = float(ref["drdT"] @ ref["r"])
    eta0, _ = W.initial_state(w)
    out = dict(r=ref["r"], J=ref["J"], drdT=ref["drdT"], f=np.array(ref["f"]), grad=grad, dfdT=np.array(dfdT),
               Jnorms=np.linalg.norm(ref["J"], axis=0), eta0max=np.array(np.abs(eta0).max()))
    alts = [t for t in ALTS if _load_raw(name, t) is not None]
    out["alt_names"] = np.array(alts)
    for key in ("r", "f", "drdT", "grad", "Jfro"):
        out[f"alt_{key}"] = np.array([_diffs(_load_raw(name, t), ref)[key] for t in alts])
    out["alt_Jcol"] = np.array([_diffs(_load_raw(name, t), ref)["Jcol"] for t in alts]).reshape(len(alts), -1)
    ddr = _load_raw(name, "dd") if name in DD_SPLIT else None
    if ddr is not None:
        d = _diffs(ref, ddr)
        for key in ("r", "f", "drdT", "grad", "Jfro", "Jcol"):
            out[f"dd_{key}"] = np.array(d[key])
        np.savez_compressed(os.path.join(HERE, f"{name}_dd.npz"), r=ddr["r"], J=ddr["J"], drdT=ddr["drdT"],
                            f=np.array(ddr["f"]))
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), **out)
    print(name, "combined: alternates", alts, "dd", ddr is not None, flush=True)


def jobs_of(name):
    js = [(name, "f64", None)] + [(name, t, None) for t in ALTS]
    sp = _splits(name)
    if sp:
        js += [(name, "dd", c if len(sp) > 1 else None) for c in sp]
    return js


def run_all(names, nproc):
    # runs already stored are kept
    jobs = [j for n in names for j in jobs_of(n) if not os.path.exists(_raw_path(*j))]
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    running = []
    while jobs or running:
        while jobs and len(running) < nproc:
            n, t, c = jobs.pop(0)
            args = [sys.executable, os.path.abspath(__file__), "run", n, t] + ([f"{c[0]}:{c[1]}"] if c else [])
            running.append(subprocess.Popen(args, env=env, cwd=ROOT))
        time.sleep(2)
        for p in list(running):
            if p.poll() is not None:
                running.remove(p)
                if p.returncode:
                    raise SystemExit(f"job {p.args} failed with {p.returncode}")
    for n in names:
        combine(n)


if __name__ == "__main__":
    a = sys.argv[1:]
    if not a:
        raise SystemExit(__doc__)
    if a[0] == "run":
        cols = tuple(int(v) for v in a[3].split(":")) if len(a) > 3 else None
        run(a[1], a[2], cols)
    elif a[0] == "combine":
        for n in a[1:]:
            combine(n)
    elif a[0] == "all":
        nproc = 7
        rest = a[1:]
        if rest[:1] == ["-j"]:
            nproc = int(rest[1])
            rest = rest[2:]
        run_all(rest or list(ALL), nproc)
    else:
        raise SystemExit(__doc__)
