"""Discrete adjoint (shoot_adjoint) against J^T r of the oracle and of the GPU's own
forward Jacobian, dfdT = r.drdT, and the autograd wrapper."""
import math
import os

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


def _small(N=48, M=4, h=1.0, tau=0.01, nsteps=8):
    p = np.array([0.05, 0.01, -0.004, 0.002])[:M]
    T = W.linear_period(h, tau)
    return W.Workload("adj", N, h, tau, 1.0, M, T, nsteps, p, W.cosine_basis(N, M), np.zeros(2 * N))


@pytest.mark.parametrize("ckpt", [3, 8, 1])
def test_adjoint_small_against_oracle(ckpt):
    ww, torch = _ww()
    w = _small()
    print(f"adjoint small ckpt={ckpt}", flush=True)
    ctx = ww.Context(n_max=64, r_max=w.M + 1)
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    out = ctx.shoot_adjoint(ww.to_dev(w.params), w.T, w.nsteps, ckpt)
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps)
    g_ref, dfdT_ref = O.shoot_gradient(ref)
    g = out["grad"].cpu().numpy()
    eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    ef = abs(out["f"] - ref["f"]) / ref["f"]
    print(eg, ef, out["dfdT"], dfdT_ref)
    assert eg < TOL and ef < TOL
    assert abs(out["dfdT"] - dfdT_ref) < 1e-10 * abs(dfdT_ref) + 1e-13


def test_adjoint_padded_grid_paper_basis():
    """N = 96 (padded to 128 internally), infinite depth, the paper's parametrisation."""
    ww, torch = _ww()
    N, M = 96, 3
    p = np.array([0.03, 0.004, -0.002])
    w = W.Workload("adjp", N, math.inf, 0.0, 1.0, M, 2 * math.pi, 10, p, W.paper_basis(N, M), np.zeros(2 * N))
    ctx = ww.Context(n_max=N, r_max=M + 1)
    ctx.shoot_setup(N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    out = ctx.shoot_adjoint(ww.to_dev(p), w.T, w.nsteps, 4)
    ref = O.shoot_eval(N, w.h, w.tau, w.g, w.basis, w.q_fixed, p, w.T, w.nsteps)
    g_ref, _ = O.shoot_gradient(ref)
    eg = np.linalg.norm(out["grad"].cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    print("padded", eg)
    assert eg < TOL


def test_adjoint_config4_full_against_forward_jacobian():
    """Differentiation form: N = 512, 256 parameters, 800 steps, checkpoints every 16:
    adjoint gradient against J^T r of the GPU forward Jacobian and of the oracle."""
    ww, torch = _ww()
    w = W.c4()
    print("adjoint c4", flush=True)
    ctx = ww.Context(n_max=w.N, r_max=w.M + 1)
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params)
    out = ctx.shoot_adjoint(p, w.T, w.nsteps, w.ckpt_every)
    fwd = ctx.shoot_eval(p, w.T, w.nsteps)
    g_fwd = (fwd["J"].t() @ fwd["r"]).cpu().numpy()
    g = out["grad"].cpu().numpy()
    e_self = np.linalg.norm(g - g_fwd) / np.linalg.norm(g_fwd)
    fx_path = os.path.join(os.path.dirname(__file__), "golden", "c4_oracle.npz")
    e_or = None
    if os.path.exists(fx_path):
        fx = np.load(fx_path)
        e_or = np.linalg.norm(g - fx["grad"]) / np.linalg.norm(fx["grad"])
    print("c4 adjoint vs forward J^T r", e_self, "vs oracle", e_or, flush=True)
    assert e_self < TOL
    if e_or is not None:
        assert e_or < TOL


def test_autograd_wrapper_and_central_difference():
    ww, torch = _ww()
    from paper_1210_5672_amd.autograd import shoot_objective
    w = _small(N=32, nsteps=6)
    ctx = ww.Context(n_max=64, r_max=w.M + 1)
    ctx.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params).requires_grad_(True)
    f = shoot_objective(p, ctx, w.T, w.nsteps, 2)
    f.backward()
    g = p.grad.cpu().numpy()
    eps = 1e-6
    fd = []
    for k in range(w.M):
        d = np.zeros(w.M)
        d[k] = eps
        fp = ctx.shoot_eval(ww.to_dev(w.params + d), w.T, w.nsteps, jacobian=False)["f"]
        fm = ctx.shoot_eval(ww.to_dev(w.params - d), w.T, w.nsteps, jacobian=False)["f"]
        fd.append((fp - fm) / (2 * eps))
    fd = np.array(fd)
    e = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    print("autograd vs FD", e)
    assert e < 1e-6
