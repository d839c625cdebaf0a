"""The lagged-factor march (the default for one instance; WW_PIPE_LAG sets the lag) in
its per-branch-graph form: every stage's base chain solves with the factors of the stage
`lag` stages earlier, refined against its own matrix, while its own LU runs on one of the
LU streams (WW_LU_STREAMS); each branch of a stage is a graph of its own, replayed on its
own stream.  Held against the oracle, against the march that solves every stage with its
own factors, and against itself under other stream layouts."""
import math

import numpy as np
import pytest

from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _ww():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5672_amd import ww
    return ww, torch


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _run(ww, w, lag, mixed=False):
    import os
    old = os.environ.get("WW_PIPE_LAG")
    os.environ["WW_PIPE_LAG"] = str(lag)
    try:
        ctx = ww.Context(n_max=max(w.N, 64), r_max=w.M + 1, mixed=mixed)
    finally:
        if old is None:
            del os.environ["WW_PIPE_LAG"]
        else:
            os.environ["WW_PIPE_LAG"] = old
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    out = ctx.shoot_eval(ww.to_dev(w.params), w.T, w.nsteps)
    return ctx, out


@pytest.mark.parametrize("lag", [2, 4])
@pytest.mark.parametrize("mixed", [False, True])
def test_lagged_march_c1(lag, mixed):
    """C1 (64 steps): ||A_old^{-1} A_new - I|| is about 6e-6 per step, so the lagged
    solves converge in the two sweeps: no fallback, the oracle's r and J to 1e-12, and
    the direct march's to 1e-12."""
    ww, torch = _ww()
    w = W.c1()
    print(f"lagged march c1 lag={lag} mixed={mixed}", flush=True)
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps)
    ctx, out = _run(ww, w, lag, mixed)
    assert ctx.fallbacks() == 0
    assert relerr(out["r"].cpu().numpy(), ref["r"]) < TOL
    assert relerr(out["J"].cpu().numpy(), ref["J"]) < TOL
    assert abs(out["f"] - ref["f"]) <= TOL * ref["f"]
    ctx0, out0 = _run(ww, w, 0, mixed)
    assert relerr(out["J"].cpu().numpy(), out0["J"].cpu().numpy()) < TOL


def test_lagged_march_falls_back_on_a_fast_changing_surface():
    """The steep surface changes too fast for factors four stages old (0.03 to 0.13 per
    step): the first step's check sends the march to each stage's own factors
    (WW_FB_DIRECT), which match the oracle; later marches on the context start there."""
    ww, torch = _ww()
    N, M = 64, 3
    eta = W.steep_surface(N)
    w = W.Workload("t", N, 1.0, 0.0, 1.0, M, 0.1, 4, np.array([0.01, 0.005, 0.002]), W.cosine_basis(N, M),
                   np.concatenate([eta, np.zeros(N)]))
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps)
    ctx, out = _run(ww, w, 4)
    assert ctx.fallbacks() == ww.WW_FB_DIRECT
    assert relerr(out["r"].cpu().numpy(), ref["r"]) < TOL
    assert relerr(out["J"].cpu().numpy(), ref["J"]) < TOL
    # the context's next march starts on each stage's own factors (the same march again,
    # so bitwise the same results); shoot_setup forgets it, and the march falls back anew
    out2 = ctx.shoot_eval(ww.to_dev(w.params), w.T, w.nsteps)
    assert ctx.fallbacks() == ww.WW_FB_DIRECT
    assert np.array_equal(out2["r"].cpu().numpy(), out["r"].cpu().numpy())
    assert np.array_equal(out2["J"].cpu().numpy(), out["J"].cpu().numpy())
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    out3 = ctx.shoot_eval(ww.to_dev(w.params), w.T, w.nsteps)
    assert ctx.fallbacks() == ww.WW_FB_DIRECT
    assert np.array_equal(out3["r"].cpu().numpy(), out["r"].cpu().numpy())
    # a WW_STRICT context reports the failure on every march (it remembers nothing)
    import os
    old = os.environ.get("WW_PIPE_LAG")
    os.environ["WW_PIPE_LAG"] = "4"
    try:
        cs = ww.Context(n_max=64, r_max=M + 1, strict=True)
    finally:
        if old is None:
            del os.environ["WW_PIPE_LAG"]
        else:
            os.environ["WW_PIPE_LAG"] = old
    cs.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    for _ in range(2):
        with pytest.raises(ww.WWError) as ei:
            cs.shoot_eval(ww.to_dev(w.params), w.T, w.nsteps)
        assert ei.value.name == "WW_EREFINE"


def test_phase_profile_in_the_lagged_march():
    """ww_profile's timestamp nodes sit inside the per-branch graphs (the LU phase on the
    LU streams, the base and column chains on theirs): every phase reads a positive mean."""
    ww, torch = _ww()
    w = W.c1()
    import os
    old = os.environ.pop("WW_PIPE_LAG", None)
    try:
        ctx = ww.Context(n_max=64, r_max=w.M + 1)
    finally:
        if old is not None:
            os.environ["WW_PIPE_LAG"] = old
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    ctx.profile(True)
    # 24 steps: the lagged solves converge (with 6 steps the stages change so fast that
    # lagged factors fail their test and the march runs on each stage's own factors)
    ctx.shoot_eval(ww.to_dev(w.params), w.T, 24)
    ph = [ctx.profile_read(k) for k in range(4)]
    print("phases ms", ph)
    assert all(p > 0 for p in ph)
    assert ctx.fallbacks() == 0


def test_block_lu_step_events():
    """Kernel events (ww_profile bit 2, phase 4): every block-LU step launched directly
    is timed, nb - 1 launches per LU sequence; none while the LU is replayed from graphs."""
    ww, torch = _ww()
    w = W.c2()
    nsteps = 24
    T = w.T * nsteps / w.nsteps
    nb = w.N // 64
    for parts, timed in ((0, True), (10, False)):
        ctx = ww.Context(n_max=w.N, r_max=w.M + 1)
        ctx.set_tuning(graph_parts=parts)
        ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        ctx.profile(True, kernel_events=True)
        ctx.shoot_eval(ww.to_dev(w.params), T, nsteps)
        seq_ms, seq_n = ctx.profile_stats(0)
        print("graph_parts", parts, "sequences", seq_n, "mean", seq_ms, flush=True)
        assert ctx.fallbacks() == 0 and seq_n > 0
        if timed:
            step_ms, step_n = ctx.profile_stats(4)
            print("step launches", step_n, "mean ms", step_ms, flush=True)
            assert step_n == (nb - 1) * seq_n
            assert 0 < step_ms < seq_ms
        else:
            with pytest.raises(ww.WWError):
                ctx.profile_stats(4)
        ctx.profile(False)
        ctx.close()


def _ctx_env(ww, n_max, r_max, env):
    """A context created under the given environment variables (read by ww_create)."""
    import os
    old = {v: os.environ.get(v) for v in env}
    os.environ.update({v: str(x) for v, x in env.items()})
    try:
        return ww.Context(n_max=n_max, r_max=r_max)
    finally:
        for v, x in old.items():
            if x is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = x


def _c2_short(M=16, nsteps=20):
    w2 = W.c2()
    return W.Workload("c2_short", w2.N, w2.h, w2.tau, w2.g, M, w2.T * nsteps / w2.nsteps, nsteps, w2.params[:M],
                      W.cosine_basis(w2.N, M), w2.q_fixed)


def test_lagged_march_is_bitwise_independent_of_the_lu_streams():
    """The lagged march's arithmetic does not depend on how its branches are scheduled:
    with 1, 2 or 5 LU streams (WW_LU_STREAMS), with the column chains on the LU streams
    (WW_COLS_ON_LU) and on a second evaluation by the same context, r and J are bitwise
    the same.  N = 256 (four 64-blocks) and 20 steps, so
    that the LUs of different stages and the split step end really overlap; a missing
    dependency between the streams would show as a difference."""
    ww, torch = _ww()
    w = _c2_short()
    N, M = w.N, w.M
    outs = []
    for k, col_on_lu in ((1, 0), (2, 0), (5, 0), (2, 1), (3, 1)):
        print(f"lagged march N=256 M=16 lag=5 LU streams={k} columns on LU streams={col_on_lu}", flush=True)
        ctx = _ctx_env(ww, N, M + 1, {"WW_PIPE_LAG": 5, "WW_LU_STREAMS": k, "WW_COLS_ON_LU": col_on_lu})
        ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        for rep in range(2):
            out = ctx.shoot_eval(ww.to_dev(w.params), w.T, w.nsteps)
            assert ctx.fallbacks() == 0
            outs.append((out["r"].cpu().numpy(), out["J"].cpu().numpy()))
        del ctx
    r0, J0 = outs[0]
    assert np.isfinite(J0).all() and np.abs(J0).max() > 0
    for r, J in outs[1:]:
        assert np.array_equal(r, r0)
        assert np.array_equal(J, J0)


def test_lagged_march_without_columns():
    """A march without Jacobian columns (the residual evaluations of the LM driver) also
    solves on lagged factors.  Its base chain is the same arithmetic as in the march with
    columns, so on one context r and f are bitwise those of the march with columns, in
    either order (the first f-only march's graphs lack the column branches, which the
    march with columns then adds); r is within 1e-12 of the march on every stage's own
    factors (lag 0) and of the oracle; no fallback."""
    ww, torch = _ww()
    w = _c2_short()
    N, M = w.N, w.M
    print("lagged march without columns N=256 M=16 lag=5", flush=True)
    ctx = _ctx_env(ww, N, M + 1, {"WW_PIPE_LAG": 5})
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params)
    outs = [ctx.shoot_eval(p, w.T, w.nsteps, jacobian=False)]
    assert ctx.fallbacks() == 0
    outs.append(ctx.shoot_eval(p, w.T, w.nsteps))
    assert ctx.fallbacks() == 0
    outs.append(ctx.shoot_eval(p, w.T, w.nsteps, jacobian=False))
    assert ctx.fallbacks() == 0
    r0 = outs[0]["r"].cpu().numpy()
    for o in outs[1:]:
        assert np.array_equal(o["r"].cpu().numpy(), r0)
        assert o["f"] == outs[0]["f"]
        assert np.array_equal(o["drdT"].cpu().numpy(), outs[0]["drdT"].cpu().numpy())
    print("lag 0 without columns", flush=True)
    ctx0 = _ctx_env(ww, N, M + 1, {"WW_PIPE_LAG": 0})
    ctx0.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    out0 = ctx0.shoot_eval(p, w.T, w.nsteps, jacobian=False)
    assert relerr(r0, out0["r"].cpu().numpy()) < TOL
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps)
    assert relerr(r0, ref["r"]) < TOL


def test_lagged_march_without_graphs_matches_the_graphs():
    """WW_NO_GRAPH=1 enqueues the same kernels in the same order on the same streams
    directly instead of replaying the per-branch graphs: r, J and the f-only r are
    bitwise the graphed march's."""
    ww, torch = _ww()
    w = _c2_short(M=8, nsteps=12)
    N, M = w.N, w.M
    outs = []
    for env in ({"WW_PIPE_LAG": 5}, {"WW_PIPE_LAG": 5, "WW_NO_GRAPH": 1}):
        print(f"lagged march N=256 M=8 {env}", flush=True)
        ctx = _ctx_env(ww, N, M + 1, env)
        ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        p = ww.to_dev(w.params)
        a = ctx.shoot_eval(p, w.T, w.nsteps)
        assert ctx.fallbacks() == 0
        b = ctx.shoot_eval(p, w.T, w.nsteps, jacobian=False)
        assert ctx.fallbacks() == 0
        outs.append((a["r"].cpu().numpy(), a["J"].cpu().numpy(), b["r"].cpu().numpy()))
        del ctx
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)
    assert np.array_equal(outs[0][0], outs[0][2])
