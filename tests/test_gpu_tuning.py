"""Launch and scheduling choices (ww_get_tuning / ww_set_tuning) and the autotuner on
the GPU: every alternative choice leaves the march's results at the oracle's bounds
(full C2 march against its stored oracle run, every column of J), invalid choices are
refused, and a short tuning run stores an entry that a context can apply."""
import os

import numpy as np
import pytest

from paper_1210_5672_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# alternatives of every choice, and combinations
ALTERNATIVES = [
    {"blu_strip": 2}, {"blu_strip": 8}, {"dtn_rows": 16}, {"dtn_rows": 4}, {"gemm_split": 2},
    {"asm_cw": 32}, {"gemm_rows": 16}, {"gemm_rows": 16, "gemm_split": 2}, {"lu_group": 1},
    {"lu_group": 3, "lu_streams": 2}, {"graph_parts": 0}, {"graph_parts": 15}, {"lag": 6}, {"minv_wgs": 64},
    {"lag_fp32": 1}, {"lag_fp32": 1, "lag": 6, "graph_parts": 0}, {"lag_sweeps": 3},
    {"blu_strip": 3, "gemm_split": 2, "asm_cw": 32, "dtn_rows": 4, "graph_parts": 0},
]


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tuning_defaults_and_validation():
    _need_gpu()
    from paper_1210_5672_amd import ww
    ctx = ww.Context(n_max=256, r_max=65)
    t = ctx.tuning()
    assert t == {"lag": 8, "lu_group": 2, "lu_streams": 3, "graph_parts": 10, "minv_wgs": 1 << 20,
                 "blu_strip": 4, "dtn_rows": 8, "gemm_split": 4, "asm_cw": 16,
                 "gemm_rows": 32, "lag_fp32": 0, "lag_sweeps": 2}, t
    for bad in ({"lag": 12}, {"lu_group": 0}, {"lu_streams": 7}, {"graph_parts": 16}, {"minv_wgs": 0},
                {"blu_strip": 17}, {"dtn_rows": 6}, {"dtn_rows": 36}, {"gemm_split": 3}, {"asm_cw": 24},
                {"gemm_rows": 8}, {"lag_fp32": 2}, {"lag_sweeps": 0}, {"lag_sweeps": 9}):
        with pytest.raises(ww.WWError) as e:
            ctx.set_tuning(**bad)
        assert e.value.name == "WW_EINVAL", bad
    assert ctx.tuning() == t   # a refused set changes nothing
    ctx.set_tuning(blu_strip=6, asm_cw=32)
    assert ctx.tuning() == dict(t, blu_strip=6, asm_cw=32)
    ctx.close()


@pytest.mark.parametrize("choices", ALTERNATIVES, ids=lambda c: ",".join(f"{k}={v}" for k, v in c.items()))
def test_alternative_choices_keep_parity(choices):
    """Full C2 march (N = 256, M = 64, 300 steps) under one set of choices against the
    stored oracle run, with the bounds of the full-size parity tests."""
    _need_gpu()
    import test_gpu_fullsize as F
    from paper_1210_5672_amd import ww
    fx = F._load("c2")
    w = W.c2()
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1)
    ctx.set_tuning(**choices)
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    print("choices", ctx.tuning(), flush=True)
    res = F._np(ctx.shoot_eval(ww.to_dev(w.params), w.T, w.nsteps))
    assert ctx.fallbacks() == 0
    F.check(fx, w, res)
    ctx.close()


def test_autotune_stores_and_applies(tmp_path):
    """A short tuning run over a reduced space on C1 writes a cache entry for this GPU's
    architecture; apply() gives a new context exactly those choices."""
    _need_gpu()
    from paper_1210_5672_amd import autotune as A
    from paper_1210_5672_amd import ww
    w = W.c1()
    space = {"blu_strip": [4, 2], "gemm_split": [4, 2], "dtn_rows": [8, 16]}
    saved = A.SPACE
    try:
        A.SPACE = space
        best, t, hist = A.tune(w, nsteps=4, reps=1, passes=1, log=lambda *a: None)
    finally:
        A.SPACE = saved
    assert t > 0 and len(hist) == 1 + sum(len(v) - 1 for v in space.values())
    p = str(tmp_path / "cache.json")
    A.store(A.key(w.N, w.M, False), best, t, "test", p)
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1)
    got = A.apply(ctx, w.N, w.M, p)
    assert got == best and ctx.tuning() == best
    ctx.close()
