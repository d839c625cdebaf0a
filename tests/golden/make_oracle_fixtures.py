"""Write full-size reference results of the CPU oracle for the parity tests.

Calls only oracle/ (and the seeded input generators).  Run from the repository root:
    python tests/golden/make_oracle_fixtures.py [c2] [c4] [c3] [c5_16x3] [c5_02x3] [alt]
With "alt", the runs use the oracle's alternative rounding of cosh/sinh (same formulas)
and are written to <name>_oracle_alt.npz: the spread between the two oracle runs is the
FP64 rounding floor of the march, to which the GPU path is compared.
Each fixture stores r, drdT, f, J^T r (the gradient of f), the column norms of J and a
sample of J columns, for the workload of the same name.  C3 takes about an hour on
8 cores (7200 dense DtN solves at N = 1024).  c5_16x3 and c5_02x3 are 3-step prefixes
of two batched instances at N = 2048 and N = 1536 (finite depth, tension).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ww_oracle as O                 # noqa: E402
from paper_1210_5672_amd import workloads as W   # noqa: E402

SAMPLE_COLS = {"c2": [0, 1, 2, 7, 15, 31, 63], "c3": [0, 1, 2, 15, 40, 63, 127],
               "c4": [0, 1, 2, 15, 63, 127, 200, 255],
               "c5_16x3": [0, 1, 2, 15, 40, 85], "c5_02x3": [0, 1, 7, 20, 39]}

# prefixes of batched continuation instances at the largest sizes: (instance, steps);
# the march uses the instance's own dt (T scaled with the step count)
C5_PREFIX = {"c5_16x3": (16, 3), "c5_02x3": (2, 3)}


def workload(name):
    if name in C5_PREFIX:
        idx, steps = C5_PREFIX[name]
        w = W.c5()[idx]
        return W.Workload(name, w.N, w.h, w.tau, w.g, w.M, w.T * steps / w.nsteps, steps, w.params, w.basis,
                          w.q_fixed, description=f"first {steps} steps of batched instance {idx}")
    return W.CONFIGS[name]()


def make(name, alt=False):
    w = workload(name)
    t0 = time.time()
    ar = O.F64ALT if alt else O.F64
    res = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps, ar=ar)
    grad, dfdT = O.shoot_gradient(res)
    cols = np.array(SAMPLE_COLS[name])
    out = os.path.join(HERE, f"{name}_oracle{'_alt' if alt else ''}.npz")
    eta0, _ = W.initial_state(w)
    np.savez_compressed(out, r=res["r"], drdT=res["drdT"], f=np.array(res["f"]), grad=grad,
                        dfdT=np.array(dfdT), Jcols=res["J"][:, cols], cols=cols,
                        Jnorms=np.linalg.norm(res["J"], axis=0), eta0max=np.array(np.abs(eta0).max()),
                        seconds=np.array(time.time() - t0))
    print(name, "done in", time.time() - t0, "s ->", out, flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    alt = "alt" in args
    names = [a for a in args if a != "alt"] or ["c2", "c4", "c3"]
    for n in names:
        make(n, alt=alt)
