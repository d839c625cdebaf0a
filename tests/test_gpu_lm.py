"""Thin SVD and the Levenberg-Marquardt driver (App. C) on the GPU against the oracle,
through the C ABI.

The SVD is held against LAPACK's (NumPy) on what is unique: the singular values, and
U S V^T = A with orthonormal U and V (the singular vectors are unique only up to sign,
or to a rotation within a repeated singular value).  The driver is held against the
oracle driver step by step: the same accept / reject decisions and the same iterates
while f is above the rounding regime, and a final point of the same quality."""
import math

import numpy as np
import pytest

from oracle import lm_oracle as L
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


def _grid_size(N):
    """Smallest even 2^a 3^b >= max(N, 16) (the context's n_max)."""
    m = max(N, 16)
    while True:
        k = m
        while k % 2 == 0:
            k //= 2
        while k % 3 == 0:
            k //= 3
        if k == 1 and m % 2 == 0:
            return m
        m += 1


def _spectrum_matrix(N, n, sv, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((N, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return U @ np.diag(sv) @ V.T


def _check_svd(ww, ctx, A):
    N, n = A.shape
    sig, V, U = ctx.thin_svd(ww.to_dev(A), want_u=True)
    U = U.cpu().numpy()
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.abs(sig - ref).max() <= TOL * ref[0], (sig[:4], ref[:4])
    assert np.all(np.diff(sig) <= 0)
    rec = U @ np.diag(sig) @ V.T
    assert np.abs(rec - A).max() <= TOL * np.abs(A).max()
    assert np.abs(V.T @ V - np.eye(n)).max() <= TOL
    nz = sig > n * 2.2e-16 * sig[0]
    Un = U[:, nz]
    assert np.abs(Un.T @ Un - np.eye(nz.sum())).max() <= TOL
    return sig


@pytest.mark.parametrize("N,n", [(300, 40), (257, 33), (64, 64), (100, 1), (1024, 129)])
def test_thin_svd_against_lapack(N, n):
    ww, torch = _ww()
    print(f"thin svd N={N} n={n}", flush=True)
    ctx = ww.Context(n_max=_grid_size(N), r_max=n)
    sv = np.geomspace(1.0, 1e-6, n) if n > 1 else np.array([2.5])
    if n > 4:
        sv[1] = sv[2] = 0.5          # a repeated singular value
    _check_svd(ww, ctx, _spectrum_matrix(N, n, sv, seed=N + n))


def test_thin_svd_rank_deficient_and_of_a_jacobian():
    ww, torch = _ww()
    N, n = 128, 12
    ctx = ww.Context(n_max=N, r_max=n)
    A = _spectrum_matrix(N, n, np.geomspace(2.0, 1e-3, n), seed=9)
    A[:, 5] = 0.0                                     # an exact zero column
    sig = _check_svd(ww, ctx, A)
    assert sig[-1] == 0.0
    # the shooting Jacobian [dr/dT | dr/dc] of the C1 workload (from the oracle)
    w = W.c1()
    ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, 16)
    J = np.concatenate([ref["drdT"][:, None], ref["J"]], axis=1)
    c2 = ww.Context(n_max=64, r_max=J.shape[1])
    _check_svd(ww, c2, J)


def test_thin_svd_largest_size():
    ww, torch = _ww()
    N, n = 2048, 257
    print(f"thin svd N={N} n={n}", flush=True)
    ctx = ww.Context(n_max=N, r_max=n)
    _check_svd(ww, ctx, _spectrum_matrix(N, n, np.geomspace(1.0, 1e-4, n), seed=3))


def _standing_wave(N, nsteps, a1, nmodes):
    """eq. (init:stand) (reading R4): eta even, phi odd modes, basis 2 cos(k alpha);
    c_1 = phi^_1 fixed; unknowns T and c_2..c_nmodes; infinite depth, g = 1."""
    a = 2 * np.pi * np.arange(N) / N
    ks = list(range(2, nmodes + 1))
    basis = np.zeros((2 * N, len(ks)))
    for j, k in enumerate(ks):
        basis[(0 if k % 2 == 0 else N):(N if k % 2 == 0 else 2 * N), j] = 2 * np.cos(k * a)
    qf = np.concatenate([np.zeros(N), 2 * a1 * np.cos(a)])
    return basis, qf, np.concatenate([[2 * np.pi], np.zeros(len(ks))])


@pytest.mark.parametrize("a1", [1e-3, 0.05])
def test_levmar_against_the_oracle_driver(a1):
    ww, torch = _ww()
    N, nsteps, nmodes = 64, 32, 10
    basis, qf, c0 = _standing_wave(N, nsteps, a1, nmodes)
    print(f"levmar standing wave a1={a1}", flush=True)

    def jac(c):
        out = O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=True)
        return out["r"], np.concatenate([out["drdT"][:, None], out["J"]], axis=1)

    def res(c):
        return O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=False)["r"]

    ref = L.levmar(res, jac, c0, delta0=0.1, max_evals=60)
    ctx = ww.Context(n_max=N, r_max=nmodes)
    ctx.shoot_setup(N, math.inf, 0.0, 1.0, ww.to_dev(basis), ww.to_dev(qf))
    out = ctx.levmar(c0, nsteps, opts={"delta0": 0.1, "max_evals": 60}, hist_cap=64)
    print("oracle", ref.f, ref.reason, ref.evals_r, ref.evals_J, "gpu", out["f"], out["reason"],
          out["evals_r"], out["evals_J"])
    assert out["f"] < 1e-26 and ref.f < 1e-26
    # the same decisions, and the same iterates while f is well above the rounding of
    # the residual (r ~ 1e-6): below that, f carries the absolute rounding of r
    for k, (cn, fn, acc, _) in enumerate(ref.history):
        if fn < 1e-20:
            break
        h = out["history"][k]
        assert bool(h[-1]) == acc, k
        if fn > 1e-12:
            assert np.abs(h[:-2] - cn).max() <= 1e-10 * np.abs(cn).max(), (k, h[:-2] - cn)
            assert abs(h[-2] - fn) <= 1e-8 * fn, (k, h[-2], fn)
    # what is unique: the period; the high modes are fixed only to within the conditioning
    # of J, so the GPU's point is checked for being a solution by the oracle itself
    assert abs(out["c"][0] - ref.c[0]) <= 1e-11 * ref.c[0]
    assert 0.5 * float(np.sum(res(out["c"]) ** 2)) < 1e-24


def test_bfgs_against_the_oracle_driver():
    """BFGS with the discrete adjoint gradient (GPU) against the oracle's BFGS with the
    gradient J^T r of the forward Jacobian (the same gradient to rounding, reading R9):
    the same iterates while f is well above the rounding of r (f > 1e-12: below that the
    gradient carries the absolute rounding of r, and the two drivers part), the same
    period, and a final point that is a solution for the oracle too."""
    from oracle import bfgs_oracle as B
    ww, torch = _ww()
    N, nsteps, nmodes, a1 = 32, 12, 10, 0.05
    basis, qf, c0 = _standing_wave(N, nsteps, a1, nmodes)

    def fg(c):
        out = O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=True)
        J = np.concatenate([out["drdT"][:, None], out["J"]], axis=1)
        return 0.5 * float(out["r"] @ out["r"]), J.T @ out["r"]

    ref = B.bfgs(fg, c0, delta0=0.1, max_iter=80)
    ctx = ww.Context(n_max=64, r_max=nmodes)
    ctx.shoot_setup(N, math.inf, 0.0, 1.0, ww.to_dev(basis), ww.to_dev(qf))
    out = ctx.bfgs(c0, nsteps, opts={"delta0": 0.1, "max_iter": 80, "ckpt_every": 4}, hist_cap=100)
    print("oracle", ref.f, ref.reason, len(ref.history), ref.evals, "gpu", out["f"], out["reason"], out["iters"],
          out["evals"])
    assert out["f"] < 1e-24 and ref.f < 1e-24
    compared = 0
    for k, (cn, fn) in enumerate(ref.history):
        if fn < 1e-12 or k >= len(out["history"]):
            break
        h = out["history"][k]
        assert np.abs(h[:-1] - cn).max() <= 1e-9 * np.abs(cn).max(), (k, h[:-1] - cn)
        assert abs(h[-1] - fn) <= 1e-7 * fn, (k, h[-1], fn)
        compared += 1
    assert compared >= 8
    assert abs(out["c"][0] - ref.c[0]) <= 1e-11 * ref.c[0]
    res = lambda c: O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=False)["r"]
    assert 0.5 * float(np.sum(res(out["c"]) ** 2)) < 1e-22
