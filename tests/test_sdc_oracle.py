"""Pins of the SDC15 oracle (oracle/sdc_oracle.py, Sec. 2.2): the Radau IIa nodes and
integration weights against the exactness that defines them, the order of one step on a
linear equation (15, with 10 sweeps; 4 + sweeps + 1 in general, so a wrong predictor or
sweep count shows), and agreement with the DOP853 march on a small standing wave; for the
double-double march, the 40-digit nodes and weights against their definition, one
double-double step against the exact solution of a linear equation to about 1e-30 (the
precision its weights must carry), and the base march against the FP64 march."""
import math

import numpy as np

from oracle import sdc_oracle as S
from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W


def test_radau_iia_nodes_and_weights():
    c = S.radau_iia_nodes()
    M = S.integration_matrix(c)
    assert len(c) == 8 and c[-1] == 1.0 and np.all(np.diff(c) > 0) and c[0] > 0
    b = M[-1]
    # Radau quadrature with 8 nodes: exact up to degree 14, not 15
    assert max(abs(np.dot(b, c ** k) - 1 / (k + 1)) for k in range(15)) < 1e-15
    assert abs(np.dot(b, c ** 15) - 1 / 16) > 1e-11
    # every row integrates the interpolant of degree 7 exactly
    assert max(np.abs(M @ c ** k - c ** (k + 1) / (k + 1)).max() for k in range(8)) < 1e-15


def _local_order(sweeps):
    lam = -1.0 + 2.0j
    F = lambda y: [lam * y[0]]
    errs = []
    dts = (1.2, 0.9)
    for dt in dts:
        y1 = S.sdc_step([np.array([1.0 + 0j])], F, dt, sweeps=sweeps)[0][0]
        errs.append(abs(y1 - np.exp(lam * dt)))
    return math.log(errs[0] / errs[1]) / math.log(dts[0] / dts[1]), errs


def test_local_order_of_one_step():
    p, errs = _local_order(10)
    print("10 sweeps: local order", p, errs)
    assert p > 15.0          # local error O(dt^16)
    p3, errs3 = _local_order(3)
    print("3 sweeps: local order", p3, errs3)
    assert 7.0 < p3 < 10.0   # 4 (predictor) + 3 (sweeps) + 1: local error O(dt^9)


def test_sdc_march_agrees_with_dop853():
    w = W.c1()
    M = 2
    a = S.shoot_eval_sdc(w.N, w.h, w.tau, w.g, w.basis[:, :M], w.q_fixed, w.params[:M], w.T, 8)
    b = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis[:, :M], w.q_fixed, w.params[:M], w.T, 64)
    assert np.abs(a["r"] - b["r"]).max() < 1e-11 * np.abs(b["r"]).max()
    assert np.abs(a["J"] - b["J"]).max() < 1e-11 * np.abs(b["J"]).max()


def test_nodes_and_matrix_to_40_digits():
    import mpmath
    c, M = S.nodes_and_matrix_mp()
    c64 = S.radau_iia_nodes()
    with mpmath.workdps(40):
        assert max(abs(mpmath.legendre(8, 2 * x - 1) - mpmath.legendre(7, 2 * x - 1)) for x in c[:-1]) < 1e-36
        assert max(abs(float(x) - y) for x, y in zip(c, c64)) < 1e-15
        ex = max(abs(mpmath.fsum(M[m][j] * c[j] ** k for j in range(8)) - c[m] ** (k + 1) / (k + 1))
                 for m in range(8) for k in range(8))
        assert ex < 1e-38
        # the last row: Radau quadrature, exact to degree 14
        assert max(abs(mpmath.fsum(M[7][j] * c[j] ** k for j in range(8)) - mpmath.mpf(1) / (k + 1))
                   for k in range(15)) < 1e-38


def test_double_double_step_on_a_linear_equation():
    """y' = -y: one double-double SDC15 step against exp(-dt) in mpmath.  The local error
    falls like dt^16 down to about 1e-30, which double-precision weights (about 1e-17)
    could not reach."""
    import mpmath
    from oracle import dd as D
    c, M = S.nodes_and_matrix_dd()
    F = lambda y: [y[0] * -1.0]
    errs = []
    for dt in (0.8, 0.6, 0.1):
        y1 = S.sdc_step([D.DD(np.array([1.0]))], F, D.DD(dt), c, M)[0]
        with mpmath.workdps(40):
            errs.append(abs(mpmath.mpf(float(y1.hi[0])) + mpmath.mpf(float(y1.lo[0])) - mpmath.exp(-mpmath.mpf(dt))))
    p = float(mpmath.log(errs[0] / errs[1]) / mpmath.log(mpmath.mpf(0.8) / mpmath.mpf(0.6)))
    print("local order", p, [float(e) for e in errs])
    assert p > 15.0
    assert errs[2] < 1e-28


def test_double_double_march_agrees_with_the_fp64_march():
    from oracle import dd as D
    N, steps, T = 32, 1, 2 * math.pi
    eta0 = 0.02 * np.cos(2 * np.pi * np.arange(N) / N)
    a = S.shoot_eval_sdc_dd(N, math.inf, 0.0, 1.0, D.DD(eta0), D.DD(np.zeros(N)), D.DD(T), steps)
    b = S.shoot_eval_sdc(N, math.inf, 0.0, 1.0, np.eye(2 * N)[:, :1] * 0.0, np.concatenate([eta0, np.zeros(N)]),
                         np.zeros(1), T, steps, jacobian=False)
    r = a["r"].to_float()
    assert np.abs(r - b["r"]).max() < 1e-13 * np.abs(b["r"]).max()
    assert abs(float(a["f"].hi) - b["f"]) < 1e-13 * b["f"]
