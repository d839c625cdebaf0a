"""GMRES base solves (flag WW_GMRES) of marches without Jacobian columns, against the
oracle (whose solves use LAPACK's LU), through the C ABI; and the fallback to LU
factors when GMRES does not reach the residual test."""
import math
import os

import numpy as np
import pytest

from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def _base_march(ww, w, nsteps=None, **kw):
    ctx = ww.Context(n_max=max(w.N, 64), r_max=w.M + 1, **kw)
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    out = ctx.shoot_eval(ww.to_dev(w.params), w.T, nsteps or w.nsteps, jacobian=False)
    return ctx, out


def _drdT_err(out, ref, w, eta0):
    """drdT on the scale of one right-hand-side evaluation at the march's amplitude (it
    is a near-cancellation at T/4; the FP64 parity tests use the same scale)."""
    op = max(math.exp(-36.0 * (k / (w.N / 2)) ** 36) * (w.g + w.tau * k * k) for k in range(w.N // 2))
    scale = max(np.abs(ref["drdT"]).max(), 0.25 * np.abs(eta0).max() / math.sqrt(w.N) * op)
    return float(np.abs(out["drdT"].cpu().numpy() - ref["drdT"]).max() / scale)


@pytest.mark.parametrize("case", ["c1", "padded"])
def test_gmres_base_march_against_the_oracle(case):
    ww, torch = _ww()
    if case == "c1":
        w = W.c1()
    else:
        rng = np.random.default_rng(5)
        N, M, h, tau = 96, 5, 0.7, 0.02
        p = np.zeros(M)
        p[0] = 0.04
        p[1:] = rng.normal(0, 1e-3, M - 1)
        w = W.Workload("t", N, h, tau, 1.0, M, W.linear_period(h, tau), 20, p, W.cosine_basis(N, M),
                       np.zeros(2 * N))
    print(f"gmres base march {case}", flush=True)
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps, jacobian=False)
    ctx, out = _base_march(ww, w, gmres=True)
    assert ctx.fallbacks() == 0
    e = dict(r=relerr(out["r"].cpu().numpy(), ref["r"]), f=abs(out["f"] - ref["f"]) / abs(ref["f"]),
             drdT=_drdT_err(out, ref, w, W.initial_state(w)[0]))
    print(e)
    assert max(e.values()) < TOL, e
    ctx2, out2 = _base_march(ww, w)             # the LU march, for comparison
    assert relerr(out["r"].cpu().numpy(), out2["r"].cpu().numpy()) < TOL


def test_gmres_base_march_full_size_c2():
    """The 300-step C2 march (N = 256) without columns: r and f against the stored
    oracle values of the same workload."""
    ww, torch = _ww()
    fx = np.load(os.path.join(GOLDEN, "c2_oracle.npz"))
    w = W.c2()
    print("gmres base march c2 full", flush=True)
    ctx, out = _base_march(ww, w, gmres=True)
    assert ctx.fallbacks() == 0
    assert relerr(out["r"].cpu().numpy(), fx["r"]) < TOL
    assert abs(out["f"] - float(fx["f"])) <= TOL * float(fx["f"])


def test_gmres_fallback_to_lu_factors():
    """On the steep surface GMRES needs more than 40 steps to reach the rounding level
    (oracle matrices, CPU), so the 24-step cycle fails the residual test: the march is
    redone with LU factors (WW_FB_DIRECT) and matches the oracle; strict contexts report
    WW_EREFINE."""
    ww, torch = _ww()
    N, M = 64, 3
    eta = W.steep_surface(N)
    w = W.Workload("t", N, 1.0, 0.0, 1.0, M, 0.1, 4, np.array([0.01, 0.005, 0.002]), W.cosine_basis(N, M),
                   np.concatenate([eta, np.zeros(N)]))
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps, jacobian=False)
    ctx, out = _base_march(ww, w, gmres=True)
    assert ctx.fallbacks() == ww.WW_FB_DIRECT
    assert relerr(out["r"].cpu().numpy(), ref["r"]) < TOL
    with pytest.raises(ww.WWError) as ei:
        _base_march(ww, w, gmres=True, strict=True)
    assert ei.value.name == "WW_EREFINE"


def test_levmar_with_gmres_residuals():
    """ww_levmar in a WW_GMRES context evaluates its residuals by GMRES marches and its
    Jacobians with LU factors: the same decisions and the same standing wave as with LU
    residuals."""
    ww, torch = _ww()
    N, nsteps, nmodes, a1 = 64, 32, 10, 0.05
    a = 2 * np.pi * np.arange(N) / N
    ks = list(range(2, nmodes + 1))
    basis = np.zeros((2 * N, len(ks)))
    for j, k in enumerate(ks):
        basis[(0 if k % 2 == 0 else N):(N if k % 2 == 0 else 2 * N), j] = 2 * np.cos(k * a)
    qf = np.concatenate([np.zeros(N), 2 * a1 * np.cos(a)])
    c0 = np.concatenate([[2 * np.pi], np.zeros(len(ks))])
    outs = []
    for gm in (False, True):
        ctx = ww.Context(n_max=N, r_max=nmodes, gmres=gm)
        ctx.shoot_setup(N, math.inf, 0.0, 1.0, ww.to_dev(basis), ww.to_dev(qf))
        outs.append(ctx.levmar(c0, nsteps, opts={"delta0": 0.1, "max_evals": 60}, hist_cap=64))
    lu, gm = outs
    print("lu", lu["f"], lu["evals_r"], lu["evals_J"], "gmres", gm["f"], gm["evals_r"], gm["evals_J"])
    assert gm["f"] < 1e-26
    for k in range(min(len(lu["history"]), len(gm["history"]))):
        if lu["history"][k][-2] < 1e-20:
            break
        assert lu["history"][k][-1] == gm["history"][k][-1]
    assert abs(gm["c"][0] - lu["c"][0]) <= 1e-11 * lu["c"][0]
