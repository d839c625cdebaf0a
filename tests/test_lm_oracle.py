"""Pins of the Levenberg-Marquardt oracle (App. C) against mathematics that does not
pass through its own formulas: the trust-region subproblem against bisection on
||p(lambda)|| = Delta and the normal equations (J^T J + lambda I) p = -J^T r; the
driver against least squares (lstsq) and against a zero-residual nonlinear fit with a
known solution; a small standing wave against the linear period."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import lm_oracle as L


def test_trust_subproblem_interior_and_boundary():
    rng = np.random.default_rng(1)
    s = np.sort(rng.uniform(0.01, 3.0, 12))[::-1]
    rt = rng.standard_normal(12)
    big = 10 * np.linalg.norm(rt / s)
    p, lam = L.trust_subproblem(s, rt, big)
    assert lam == 0.0
    assert np.allclose(p, -rt / s, rtol=1e-15, atol=0)
    for delta in (1e-3, 0.1, 0.5 * np.linalg.norm(rt / s)):
        p, lam = L.trust_subproblem(s, rt, delta)
        assert abs(np.linalg.norm(p) - delta) <= 1e-11 * delta
        # the root of ||p(lambda)|| - Delta by bisection (no Newton, no derivative)
        h = lambda x: np.linalg.norm(-s * rt / (s * s + x)) - delta
        lb = so.brentq(h, 0.0, 1e12, xtol=1e-15, rtol=1e-15)
        assert abs(lam - lb) <= 1e-9 * max(lb, 1.0)


def test_full_space_step_satisfies_the_normal_equations():
    rng = np.random.default_rng(2)
    J = rng.standard_normal((40, 7)) @ np.diag([3, 2, 1, 0.5, 0.1, 0.01, 1e-3])
    r = rng.standard_normal(40)
    U, s, V = L.thin_svd(J)
    delta = 0.05
    pt, lam = L.trust_subproblem(s, U.T @ r, delta)
    p = V @ pt
    assert lam > 0
    assert abs(np.linalg.norm(p) - delta) <= 1e-11 * delta
    lhs = (J.T @ J + lam * np.eye(7)) @ p
    assert np.allclose(lhs, -J.T @ r, rtol=1e-9, atol=1e-12 * np.abs(J.T @ r).max())


def test_levmar_linear_least_squares():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 5))
    cstar = rng.standard_normal(5)
    b = A @ cstar                                  # consistent: f* = 0
    res = L.levmar(lambda c: A @ c - b, lambda c: (A @ c - b, A), np.zeros(5), delta0=0.1)
    assert np.allclose(res.c, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-12, atol=1e-13)
    assert res.f < 1e-26
    b2 = b + 0.1 * rng.standard_normal(30)        # inconsistent: f* > 0
    res2 = L.levmar(lambda c: A @ c - b2, lambda c: (A @ c - b2, A), np.zeros(5), delta0=0.1)
    c2 = np.linalg.lstsq(A, b2, rcond=None)[0]
    assert np.allclose(res2.c, c2, rtol=1e-10, atol=1e-12)
    assert abs(res2.f - 0.5 * np.sum((A @ c2 - b2) ** 2)) <= 1e-12 * res2.f


def test_levmar_nonlinear_zero_residual_fit_reuses_the_jacobian():
    t = np.linspace(0, 2, 25)
    cstar = np.array([1.5, -0.7, 0.3])
    y = cstar[0] * np.exp(cstar[1] * t) + cstar[2]

    def res(c):
        return c[0] * np.exp(c[1] * t) + c[2] - y

    def jac(c):
        e = np.exp(c[1] * t)
        return res(c), np.stack([e, c[0] * t * e, np.ones_like(t)], axis=1)

    out = L.levmar(res, jac, np.array([1.0, -0.5, 0.0]), delta0=0.5)
    assert np.allclose(out.c, cstar, rtol=1e-12, atol=1e-13)
    assert out.f < 1e-26
    assert out.evals_J < out.evals_r          # delayed Jacobian updates (App. C)


def standing_wave_problem(N=32, nsteps=12, a1=1e-3, nmodes=6):
    """The paper's standing-wave parametrisation (eq. (init:stand), reading R4): eta
    even modes, phi odd modes, basis 2 cos(k alpha); c_1 = phi^_1 fixed (amplitude);
    unknowns T and c_2..c_nmodes; infinite depth, g = 1, tau = 0."""
    from oracle import ww_oracle as O
    a = 2 * np.pi * np.arange(N) / N
    ks = list(range(2, nmodes + 1))
    basis = np.zeros((2 * N, len(ks)))
    for j, k in enumerate(ks):
        if k % 2 == 0:
            basis[:N, j] = 2 * np.cos(k * a)
        else:
            basis[N:, j] = 2 * np.cos(k * a)
    qf = np.concatenate([np.zeros(N), 2 * a1 * np.cos(a)])

    def jac(c):
        out = O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=True)
        return out["r"], np.concatenate([out["drdT"][:, None], out["J"]], axis=1)

    def res(c):
        return O.shoot_eval(N, math.inf, 0.0, 1.0, basis, qf, c[1:], c[0], nsteps, jacobian=False)["r"]

    return res, jac, np.concatenate([[2 * np.pi], np.zeros(len(ks))])


def test_levmar_small_standing_wave_converges_near_the_linear_period():
    """At amplitude c_1 = 1e-3 the period differs from the linear one (2 pi) by O(c_1^2);
    the driver reaches f below 1e-26 from the linear guess."""
    res, jac, c0 = standing_wave_problem()
    out = L.levmar(res, jac, c0, delta0=0.1, max_evals=60)
    assert out.f < 1e-26, (out.f, out.reason)
    assert abs(out.c[0] - 2 * np.pi) < 1e-4
    assert np.abs(out.c[1:]).max() < 1e-5


def test_standing_wave_period_shift_is_second_order_in_amplitude():
    """The frequency of a standing wave is even in its amplitude: the period shift found
    by the driver at c_1 = 2e-3 is four times the one at 1e-3 (to 2 %)."""
    shifts = []
    for a1 in (1e-3, 2e-3):
        res, jac, c0 = standing_wave_problem(a1=a1)
        out = L.levmar(res, jac, c0, delta0=0.1, max_evals=60)
        assert out.f < 1e-24
        shifts.append(out.c[0] - 2 * np.pi)
    assert shifts[0] > 0
    assert abs(shifts[1] / shifts[0] - 4.0) < 0.08


# ----- BFGS (ACM minimiser, Sec. 3.2) -----
from oracle import bfgs_oracle as B


def test_bfgs_minimises_a_convex_quadratic_exactly():
    """On f = x^T A x / 2 - b^T x the minimiser is A^{-1} b (solve), reached to rounding."""
    rng = np.random.default_rng(4)
    Q = rng.standard_normal((6, 6))
    A = Q @ Q.T + 6 * np.eye(6)
    b = rng.standard_normal(6)
    out = B.bfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(6), f_tol=-np.inf, g_tol=1e-13)
    assert np.allclose(out.c, np.linalg.solve(A, b), rtol=1e-11, atol=1e-13)
    assert out.reason == "g_tol"


def test_bfgs_rosenbrock_reaches_the_minimum():
    """The Rosenbrock valley's unique minimiser (1, 1), against scipy's BFGS reaching it too."""
    import scipy.optimize as so

    def fg(x):
        a, b_ = x
        return (1 - a) ** 2 + 100 * (b_ - a * a) ** 2, np.array([-2 * (1 - a) - 400 * a * (b_ - a * a),
                                                                 200 * (b_ - a * a)])
    out = B.bfgs(fg, np.array([-1.2, 1.0]), delta0=1.0, f_tol=1e-24, g_tol=1e-12)
    assert np.allclose(out.c, [1.0, 1.0], atol=1e-9)
    ref = so.minimize(lambda x: fg(x)[0], np.array([-1.2, 1.0]), jac=lambda x: fg(x)[1], method="BFGS",
                      options={"gtol": 1e-10})
    assert np.allclose(ref.x, out.c, atol=1e-6)


def test_bfgs_line_search_meets_the_strong_wolfe_conditions():
    rng = np.random.default_rng(5)
    A = np.diag(rng.uniform(0.5, 5.0, 5))
    fg = lambda x: (0.5 * x @ A @ x + np.sum(np.cos(x)), A @ x - np.sin(x))
    c = rng.standard_normal(5)
    f0, g0 = fg(c)
    p = -g0
    a, f, g, _, ok = B.line_search(fg, c, f0, g0, p, 1.0)
    assert ok
    assert f <= f0 + B.C1 * a * (g0 @ p)
    assert abs(g @ p) <= -B.C2 * (g0 @ p)


def _scripted(c_star, K=None, bad_calls=()):
    """A residual whose quadratic model is exact, r(c) = [c - c*; K] with J = [I; 0],
    except on the residual calls listed in bad_calls, which return a residual far from
    the model (the step is then rejected)."""
    calls = {"n": 0}
    extra = [] if K is None else [K]

    def res(c):
        calls["n"] += 1
        r = np.concatenate([c - c_star, extra])
        if calls["n"] in bad_calls:
            r = r + 10.0
        return r

    def jac(c):
        n = len(c)
        J = np.vstack([np.eye(n), np.zeros((len(extra), n))])
        return np.concatenate([c - c_star, extra]), J

    return res, jac


def test_levmar_rule2_delta_trigger_and_radius_reset():
    """App. C rule 2 with hand-computed radii: from c = 0 toward c* = (1, 0), Delta_0 =
    0.1.  Step 1 (model exact, rho = 1, full radius) is accepted and the radius grows
    by alpha_1 to 0.1875.  Steps 2 and 3 are rejected: the first rejected radius after
    an accepted step, 0.1875, becomes delta_first_rejected, and each rejection shrinks
    the radius to alpha_0 ||p|| (0.0703125, then 0.0263672).  The second falls below
    delta_trigger = alpha_2 * 0.1875 = 0.0375, so J is recomputed and the radius reset to
    delta_first_rejected / alpha_1 = 0.1, which the fourth step uses."""
    res, jac = _scripted(np.array([1.0, 0.0]), bad_calls=(2, 3))
    out = L.levmar(res, jac, np.zeros(2), delta0=0.1, max_evals=6)
    radii = [h[3] for h in out.history]
    acc = [h[2] for h in out.history]
    assert acc[:4] == [True, False, False, True]
    assert np.allclose(radii[:4], [0.1, 0.1875, 0.0703125, 0.1], rtol=1e-14, atol=0)
    # J evaluations: the first, then the recomputation after step 3
    res2, jac2 = _scripted(np.array([1.0, 0.0]), bad_calls=(2, 3))
    out3 = L.levmar(res2, jac2, np.zeros(2), delta0=0.1, max_evals=4)
    assert (out3.evals_r, out3.evals_J) == (3, 2)
    # one rejection only: 0.0703125 stays above the trigger, J is kept, and the next
    # radius is the shrunk one
    res1, jac1 = _scripted(np.array([1.0, 0.0]), bad_calls=(2,))
    out1 = L.levmar(res1, jac1, np.zeros(2), delta0=0.1, max_evals=4)
    assert [h[3] for h in out1.history[:3]] == pytest.approx([0.1, 0.1875, 0.0703125], rel=1e-14)
    assert out1.evals_J == 1


def test_levmar_rule2_first_rejection_before_any_acceptance_is_not_remembered():
    """Reading L2: a rejection before the first accepted step of a Jacobian does not set
    delta_first_rejected, so no trigger fires however small the radius gets."""
    res, jac = _scripted(np.array([1.0, 0.0]), bad_calls=(1, 2, 3))
    out = L.levmar(res, jac, np.zeros(2), delta0=0.1, max_evals=4)
    radii = [h[3] for h in out.history]
    assert [h[2] for h in out.history] == [False, False, False]
    assert np.allclose(radii, [0.1, 0.0375, 0.0140625], rtol=1e-14, atol=0)
    assert out.evals_J == 1


def test_levmar_rule3_small_predicted_decrease_recomputes_the_jacobian():
    """App. C rule 3 (reading L3): with a constant residual part K = 100 (f ~ 5000),
    step 1 predicts |df|/f = 0.495/5000.5 ~ 1e-4 >= df_tol (no roundoff regime); step 2
    lands on the minimiser with |df|/f = 0.005/5000.005 ~ 1e-6 < df_tol, so J is
    recomputed after two residual evaluations; at the fresh J the step is zero and the
    driver stops with c unchanged, at c*."""
    res, jac = _scripted(np.array([1.0, 0.0]), K=100.0)
    out = L.levmar(res, jac, np.zeros(2), delta0=0.9)
    assert (out.evals_r, out.evals_J) == (2, 2)
    assert out.reason == "c unchanged"
    assert np.allclose(out.c, [1.0, 0.0], rtol=0, atol=1e-15)
    assert [h[2] for h in out.history] == [True, True]
    assert np.allclose([h[3] for h in out.history], [0.9, 1.6875], rtol=1e-14, atol=0)
