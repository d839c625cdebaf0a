"""Double-double DtN on the GPU (dtn_setup_dd, dtn_solve_multi_dd) against the
double-double oracle (oracle/dd.py running oracle/ww_oracle.py's DtN), element by
element, through the C ABI: infinite and finite depth, surfaces and right-hand sides
with low parts, several right-hand sides, the densities mu and G psi; plus the argument
checks.  The double-double oracle itself is pinned against mpmath by
tests/test_oracle_dd.py."""
import math

import numpy as np
import pytest

from oracle import dd as D
from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W

pytestmark = pytest.mark.gpu

# Against the double-double oracle: its exp (scaled by 2^-10, then ten squarings) is
# pinned only to 1e-28 relative, and the cot's imaginary part of near-diagonal entries
# takes sinh(y) of small y ~ 1e-3 as a difference of exponentials, which turns that into
# up to about 1e-26 on single entries of A; on G psi the two sides meet within 1e-27.
TOL = 1e-27
# Against the 40-digit mpmath oracle (the truth of the discrete operator): the GPU's own
# double-double error, sums over N terms and the derivative gamma = mu' (a factor up to
# N/2 on the rounding of mu), cond(A) <= 2
TOL_MP = 1e-30


def _ww():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5672_amd import ww
    return ww, torch


def _lo(x, seed):
    """Low parts below half an ulp of the high parts."""
    rng = np.random.default_rng(seed)
    return x * 2.0 ** -60 * rng.uniform(-1, 1, x.shape)


def _err(hi, lo, ref):
    d = D.DD(hi, lo) - ref
    return float(np.abs(d.hi).max() / np.abs(ref.hi).max())


# R = 1: the one-column products (the inner-index split of the double-double march)
@pytest.mark.parametrize("N,h,R", [(64, math.inf, 3), (64, 0.7, 5), (128, 1.5, 2), (256, math.inf, 4),
                                   (128, 0.7, 1)])
def test_dd_dtn_matches_the_dd_oracle(N, h, R):
    ww, torch = _ww()
    print(f"dd dtn N={N} h={h} R={R}", flush=True)
    eh = W.random_surface(N, seed=N + R, amp=0.06)
    el = _lo(eh, 1)
    rh = np.ascontiguousarray(W.random_rhs(N, R, seed=3 + N))
    rl = _lo(rh, 2)
    ctx = ww.Context(n_max=max(N, 64), r_max=R + 1)
    ctx.dtn_setup_dd(ww.to_dev(eh), ww.to_dev(el), h)
    oh, ol, mh, ml = ctx.dtn_solve_multi_dd(ww.to_dev(rh), ww.to_dev(rl), want_mu=True)
    torch.cuda.synchronize()
    dtn = O.DtN(D.DD(eh, el), h, ar=D.DDArith())
    ref, mref = dtn.apply(D.DD(rh, rl))
    eo = _err(oh.cpu().numpy(), ol.cpu().numpy(), ref)
    em = _err(mh.cpu().numpy(), ml.cpu().numpy(), mref)
    print(f"errors: G psi {eo:.2e}, mu {em:.2e}", flush=True)
    assert eo < TOL and em < TOL
    ctx.close()


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("h", [math.inf, 0.7])
def test_dd_dtn_against_40_digit_oracle(h, mixed):
    """The same DtN in 40-digit mpmath arithmetic (oracle/xprec.py running ww_oracle's
    DtN) at N = 64: the GPU's double-double result to 1e-30, with FP64 factors for the
    corrections or (a WW_MIXED context) FP32 factors on MFMA and more sweeps."""
    ww, torch = _ww()
    import mpmath
    from oracle import xprec
    N, R = 64, 2
    eh = W.random_surface(N, seed=5, amp=0.06)
    el = _lo(eh, 3)
    rh = np.ascontiguousarray(W.random_rhs(N, R, seed=9))
    rl = _lo(rh, 4)
    ctx = ww.Context(n_max=N, r_max=R, mixed=mixed)
    ctx.dtn_setup_dd(ww.to_dev(eh), ww.to_dev(el), h)
    oh, ol = ctx.dtn_solve_multi_dd(ww.to_dev(rh), ww.to_dev(rl))
    oh, ol = oh.cpu().numpy(), ol.cpu().numpy()
    ar = xprec.MPArith(dps=40)
    mp = ar.ctx.mpf
    eta = np.array([mp(a) + mp(b) for a, b in zip(eh, el)], dtype=object)
    psi = np.array([[mp(rh[i, c]) + mp(rl[i, c]) for c in range(R)] for i in range(N)], dtype=object)
    ref, _ = O.DtN(eta, h, ar=ar).apply(psi)
    scale = max(abs(v) for v in ref.ravel())
    err = max(abs(mp(oh[i, c]) + mp(ol[i, c]) - ref[i, c]) for i in range(N) for c in range(R)) / scale
    print(f"error against 40 digits: {float(err):.2e}", flush=True)
    assert err < TOL_MP
    ctx.close()


def test_dd_dtn_flat_surface_symbol():
    """Flat surface at finite depth: G cos(k x) = k tanh(k h) cos(k x) in double-double
    (the symbol from mpmath), the pin of the kernels' signs and factors at 32 digits."""
    ww, torch = _ww()
    import mpmath
    mpmath.mp.dps = 40
    N, h = 128, 1.0
    a = 2 * np.pi * np.arange(N) / N
    ctx = ww.Context(n_max=N, r_max=4)
    ctx.dtn_setup_dd(ww.to_dev(np.zeros(N)), None, h)
    ks = (1, 3, 7)
    # cos(k alpha_j) in double-double from mpmath
    vals = [[mpmath.cos(2 * mpmath.pi * k * j / N) for j in range(N)] for k in ks]
    hi = np.array([[float(v) for v in row] for row in vals]).T
    lo = np.array([[float(v - mpmath.mpf(float(v))) for v in row] for row in vals]).T
    oh, ol = ctx.dtn_solve_multi_dd(ww.to_dev(np.ascontiguousarray(hi)), ww.to_dev(np.ascontiguousarray(lo)))
    oh, ol = oh.cpu().numpy(), ol.cpu().numpy()
    for c, k in enumerate(ks):
        sym = k * mpmath.tanh(k * h)
        err = max(abs(mpmath.mpf(oh[j, c]) + mpmath.mpf(ol[j, c]) - sym * vals[c][j]) for j in range(N))
        print(f"k={k}: {float(err):.2e}", flush=True)
        # the flat symbol holds up to the aliasing e^{-2 (N - k) h} of the image sum
        assert err < 1e-29 + 10 * math.exp(-2 * (N - k) * h)
    ctx.close()


def test_dd_argument_checks():
    ww, torch = _ww()
    ctx = ww.Context(n_max=256, r_max=3)
    one = ww.to_dev(np.zeros((64, 1)))
    with pytest.raises(ww.WWError) as e:
        ctx.dtn_solve_multi_dd(one, None)
    assert e.value.name == "WW_ENOSETUP"
    for N in (48, 8, 512):   # not a power of two; too small; above n_max
        with pytest.raises(ww.WWError) as e:
            ctx.dtn_setup_dd(ww.to_dev(np.zeros(N)), None, math.inf)
        assert e.value.name == "WW_EINVAL", N
    with pytest.raises(ww.WWError) as e:   # finite depth, surface through the bottom
        ctx.dtn_setup_dd(ww.to_dev(np.full(64, -2.0)), None, 1.0)
    assert e.value.name == "WW_EDOMAIN"
    ctx.dtn_setup_dd(ww.to_dev(W.random_surface(64, seed=1)), None, math.inf)
    with pytest.raises(ww.WWError) as e:   # more columns than r_max
        ctx.dtn_solve_multi_dd(ww.to_dev(np.zeros((64, 4))), None)
    assert e.value.name == "WW_EINVAL"
    out = ctx.dtn_solve_multi_dd(ww.to_dev(np.ones((64, 2))), None)
    assert np.abs(out[0].cpu().numpy()).max() < 1e-12   # G of a constant is zero
    ctx.close()
