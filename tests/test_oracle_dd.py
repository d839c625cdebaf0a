"""The double-double backend of the CPU reference (oracle/dd.py) and the FP64 rounding
floor it measures (P13).

The backend is pinned against mpmath at 40-50 digits: the elementary operations and
functions, the Fourier multipliers, the dense solve and a whole short march.  Then
the FP64 reference is held against the stored double-double march of C1 (all 8
columns, 64 steps, written by tests/golden/make_oracle_fixtures.py) and, where that
run has been stored, of C2 (64 columns, 300 steps): the measured floor.  The four
alternate FP64 roundings (cosh/sinh from the math library, the full complex FFT,
reversed summation order, solves through the explicit inverse) are shown to spread
about as far as the true FP64 error,
which is what lets them stand in for the floor on the workloads too large for a
double-double run (C3, C4, the batched instances).
"""
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import dd
from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MP = mpmath.MPContext()
MP.dps = 50


def _mp(x: dd.DD):
    return [MP.mpf(float(h)) + MP.mpf(float(l)) for h, l in zip(x.hi.ravel(), x.lo.ravel())]


def _maxrel(x: dd.DD, ref):
    got = _mp(x)
    return float(max(abs(a - b) / max(abs(b), MP.mpf("1e-300")) for a, b in zip(got, ref)))


def test_dd_arithmetic_against_mpmath():
    rng = np.random.default_rng(0)
    a = dd.DD(rng.uniform(-3, 3, 300)) + dd.DD(rng.uniform(-1, 1, 300) * 1e-17)
    b = dd.DD(rng.uniform(0.5, 3, 300)) + dd.DD(rng.uniform(-1, 1, 300) * 1e-17)
    am, bm = _mp(a), _mp(b)
    assert max(abs(u - (x + y)) for u, x, y in zip(_mp(a + b), am, bm)) < 1e-31
    assert _maxrel(a * b, [x * y for x, y in zip(am, bm)]) < 3e-32
    assert _maxrel(a / b, [x / y for x, y in zip(am, bm)]) < 3e-32
    assert _maxrel(dd.sqrt(b), [MP.sqrt(y) for y in bm]) < 3e-32
    assert _maxrel(dd.exp(a), [MP.exp(x) for x in am]) < 1e-28
    x = dd.DD(rng.uniform(-13, 13, 300)) + dd.DD(rng.uniform(-1, 1, 300) * 1e-16)
    xm = _mp(x)
    s, c = dd.sin_cos(x)
    assert max(abs(u - MP.sin(v)) for u, v in zip(_mp(s), xm)) < 1e-31
    assert max(abs(u - MP.cos(v)) for u, v in zip(_mp(c), xm)) < 1e-31


def test_dd_fourier_multipliers_against_the_dft_definition():
    """d/dx, H, P and the filter in double-double against the naive DFT with the same
    symbols (k in -N/2+1..N/2, Nyquist as in the FP64 reference) in 50 digits."""
    N = 16
    rng = np.random.default_rng(1)
    f = rng.standard_normal(N)
    ar = dd.DDArith()
    ks = list(range(-N // 2 + 1, N // 2 + 1))
    a = [2 * MP.pi * j / N for j in range(N)]
    fh = {k: sum(MP.mpf(f[j]) * MP.expj(-k * a[j]) for j in range(N)) / N for k in ks}
    sym = {
        "d": lambda k: 0 if 2 * k == N else MP.mpc(0, k),
        "h": lambda k: 0 if (2 * k == N or k == 0) else MP.mpc(0, -MP.sign(k)),
        "p": lambda k: 0 if k == 0 else 1,
        "f": lambda k: MP.exp(-36 * (MP.mpf(abs(k)) / (N // 2)) ** 36),
    }
    for kind, m in sym.items():
        ref = [sum(m(k) * fh[k] * MP.expj(k * a[j]) for k in ks).real for j in range(N)]
        got = _mp(ar.spectral(kind, dd.DD(f)))
        assert max(abs(u - v) for u, v in zip(got, ref)) < 1e-29, kind


def test_dd_dense_solve_against_mpmath():
    rng = np.random.default_rng(2)
    n = 12
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal((n, 3))
    x = dd.lu_solve(dd.lu_factor(dd.DD(A)), dd.DD(b))
    Am = MP.matrix(A.tolist())
    for c in range(3):
        xm = MP.lu_solve(Am, MP.matrix(b[:, c].tolist()))
        got = _mp(x[:, c])
        assert max(abs(u - v) for u, v in zip(got, xm)) < 1e-29


def test_dd_march_against_mpmath():
    """The whole reference march (DtN, right-hand sides, filter, DOP853, outputs) in
    double-double against the same code in 40-digit mpmath, finite depth with
    tension: they agree to about 1e-28, 13 digits beyond FP64."""
    from oracle.xprec import MPArith
    mpmath.mp.dps = 50
    N, M, h, tau, nsteps = 16, 2, 1.0, 0.01, 2
    basis = W.cosine_basis(N, M)
    p = np.array([0.05, 0.01])
    ref = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, 7.0, nsteps, ar=MPArith(40))
    got = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, 7.0, nsteps, ar=dd.DDArith())
    for key in ("r", "J", "drdT"):
        rv = [mpmath.mpf(v) for v in np.ravel(ref[key])]
        gv = _mp(got[key])
        err = max(abs(a - b) for a, b in zip(gv, rv)) / max(abs(v) for v in rv)
        assert err < 1e-26, (key, float(err))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _fp64_vs_dd(res, ddr):
    return {"r": _rel(res["r"], ddr["r"]), "J": _rel(res["J"], ddr["J"]),
            "f": abs(res["f"] - float(ddr["f"])) / abs(float(ddr["f"])),
            "drdT": _rel(res["drdT"], ddr["drdT"]),
            "grad": _rel(res["J"].T @ res["r"], ddr["J"].T @ ddr["r"])}


def test_fp64_floor_at_config1_against_double_double():
    """P13 at C1: the FP64 reference against the stored double-double march, all of r,
    J, f and the gradient J^T r within 1e-13 (measured: r 5e-15, J 4e-15, f 1e-14,
    grad 9e-15).  dr/dT is one right-hand-side evaluation at the final state, which
    multiplies the final-state error by the operator scale (about k_max = 32 here):
    1e-11 (measured 3.4e-12)."""
    p = os.path.join(GOLDEN, "c1_dd.npz")
    if not os.path.exists(p):
        pytest.skip("c1 double-double run not stored")
    ddr = np.load(p)
    w = W.c1()
    res = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps)
    e = _fp64_vs_dd(res, ddr)
    print("C1 FP64 vs double-double", e)
    assert max(e[k] for k in ("r", "J", "f", "grad")) < 1e-13, e
    assert e["drdT"] < 1e-11, e


def test_alternate_roundings_bracket_the_fp64_error_at_config1():
    """Each alternate FP64 rounding differs from the reference by about as much as the
    reference differs from double-double: the largest spread over the four lies
    within a factor 10 of the true error, in r, J, f, dr/dT and the gradient, and twice
    it bounds the true error, also per column of J (there up to one rounding of the
    largest entry, 2e-16 of max |J|, where a column's spread happens to vanish)."""
    p = os.path.join(GOLDEN, "c1_dd.npz")
    if not os.path.exists(p):
        pytest.skip("c1 double-double run not stored")
    ddr = np.load(p)
    w = W.c1()
    run = lambda ar: O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps, ar=ar)
    ref = run(O.F64)
    true = _fp64_vs_dd(ref, ddr)
    spread = {k: 0.0 for k in true}
    col_true = np.abs(ref["J"] - ddr["J"]).max(axis=0)
    col_spread = np.zeros_like(col_true)
    for ar in (O.F64ALT, O.F64ALT_FFT, O.F64ALT_SUM, O.F64ALT_INV):
        alt = run(ar)
        for k, v in _fp64_vs_dd(alt, ref).items():
            spread[k] = max(spread[k], v)
        col_spread = np.maximum(col_spread, np.abs(alt["J"] - ref["J"]).max(axis=0))
    print("true FP64 error", true, "largest alternate spread", spread)
    for k in true:
        assert true[k] / 10 <= spread[k] <= 10 * true[k], (k, true[k], spread[k])
        assert true[k] <= 2 * spread[k], (k, true[k], spread[k])
    scale = np.abs(ref["J"]).max()
    assert np.all(col_true <= 2 * col_spread + 2e-16 * scale), (col_true, col_spread)


def test_fp64_floor_at_config2_against_double_double():
    """P13 at C2 (N = 256, h = 1, M = 64, 300 steps), from the stored runs.  Over 300
    steps the FP64 error itself reaches the 1e-13 level (measured against double-double:
    r 7e-15, f 8e-15, grad 1.1e-14, J 1.04e-13, dr/dT 7.5e-12), so the reference is held
    to the metric's bar, 1e-12, in r, J, f and the gradient (dr/dT: 1e-11, one
    right-hand-side evaluation at the final state), and the alternate roundings must
    bracket the true error as at C1: their largest spread within a factor 10 of it and
    twice the spread above it."""
    p = os.path.join(GOLDEN, "c2_oracle.npz")
    if not os.path.exists(p):
        pytest.skip("c2 runs not stored")
    fx = np.load(p)
    if "dd_r" not in fx.files:
        pytest.skip("c2 double-double run not stored")
    true = {k: float(fx[f"dd_{k}"]) for k in ("r", "f", "drdT", "grad", "Jfro")}
    spread = {k: float(np.max(fx[f"alt_{k}"])) for k in true}
    print("C2 FP64 vs double-double", true, "largest alternate spread", spread)
    assert max(true[k] for k in ("r", "f", "grad", "Jfro")) < 1e-12, true
    assert true["drdT"] < 1e-11, true
    for k in true:
        assert true[k] / 10 <= spread[k] <= 10 * true[k], (k, true[k], spread[k])
        assert true[k] <= 2 * spread[k], (k, true[k], spread[k])
