"""CPU reference ("oracle") for the 15th-order spectral deferred correction time
stepper of Wilkening & Yu (SDC15, Sec. 2.2): eight Radau IIa nodes, initial values at
the nodes by fourth-order Runge-Kutta from node to node, ten pure Picard correction
sweeps, and a final integration step.

TEST INFRASTRUCTURE ONLY, like oracle/ww_oracle.py (whose right-hand sides and filter
it marches); it shares no code with the GPU library.  FP64 numpy.

Reading S1 (listed with the design notes): one step from y_0 over dt is
  * predictor: classical RK4 from c_{m-1} to c_m (c_0 = 0), m = 1..8, giving Y^0_m;
  * sweep k = 1..10: Y^k_m = y_0 + dt sum_j S_mj F(Y^{k-1}_j), S_mj the integral from
    0 to c_m of the Lagrange polynomial of node j (exact Radau IIa collocation weights);
  * final integration: y_1 = y_0 + dt sum_j S_8j F(Y^10_j) (c_8 = 1);
113 evaluations of F per step (the RK4 stages, F at the last predicted node, F at the
nodes of sweeps 1..10).  The paper speaks of 99 internal stages and does not spell the
count out; the order (4 from the predictor, one per sweep, one from the final step:
local error O(dt^16)) is the one it states.  The filter is applied to every right-hand
side and to the state after every step, as for the Runge-Kutta march (reading R7).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as L

from . import ww_oracle as O

NODES = 8
SWEEPS = 10


def radau_iia_nodes(m: int = NODES) -> np.ndarray:
    """Radau IIa nodes on (0, 1]: the zeros of P_m(2c - 1) - P_{m-1}(2c - 1), with c_m = 1
    (Hairer & Wanner, Solving ODEs II, Sec. IV.5)."""
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    coef[m - 1] = -1.0
    x = np.sort(L.legroots(coef).real)
    c = (x + 1.0) / 2.0
    c[-1] = 1.0
    return c


def integration_matrix(c: np.ndarray) -> np.ndarray:
    """S[m, j] = integral from 0 to c_m of the Lagrange polynomial of node j, by 16-point
    Gauss-Legendre quadrature on [0, c_m] (exact for the degree-7 basis), the basis
    evaluated in product form."""
    m = len(c)
    xg, wg = L.leggauss(16)
    S = np.zeros((m, m))
    for i in range(m):
        x = c[i] * (xg + 1.0) / 2.0
        for j in range(m):
            ell = np.ones_like(x)
            for k in range(m):
                if k != j:
                    ell = ell * (x - c[k]) / (c[j] - c[k])
            S[i, j] = c[i] / 2.0 * np.dot(wg, ell)
    return S


def nodes_and_matrix_mp(dps: int = 40):
    """The Radau IIa nodes and the integration matrix in mpmath at `dps` digits: the
    nodes by Newton's method on P_8(x) - P_7(x) from the double-precision roots, S_mj by
    mpmath's quadrature of the Lagrange polynomial of node j over [0, c_m]."""
    import mpmath
    c0 = radau_iia_nodes()
    with mpmath.workdps(dps):
        f = lambda x: mpmath.legendre(NODES, x) - mpmath.legendre(NODES - 1, x)
        c = [(mpmath.findroot(f, mpmath.mpf(2 * ci - 1)) + 1) / 2 for ci in c0[:-1]] + [mpmath.mpf(1)]

        def ell(j):
            return lambda t: mpmath.fprod((t - c[k]) / (c[j] - c[k]) for k in range(NODES) if k != j)

        S = [[mpmath.quad(ell(j), [0, c[m]]) for j in range(NODES)] for m in range(NODES)]
        return c, S


def nodes_and_matrix_dd():
    """The nodes and the integration matrix as double-double scalars (the march in
    double-double needs its weights to about 32 digits)."""
    from . import dd as D
    c, S = nodes_and_matrix_mp()
    return [D.from_mp(v) for v in c], [[D.from_mp(v) for v in row] for row in S]


def sdc_step(y, F, dt, c=None, S=None, sweeps=SWEEPS):
    """One SDC15 step of y' = F(y) for a state given as a list of arrays (None entries
    pass through); returns the new state (unfiltered).  c, S: the nodes and the
    integration matrix (numpy, or lists of double-double scalars for a double-double
    march)."""
    c = radau_iia_nodes() if c is None else c
    S = integration_matrix(c) if S is None else S
    add = lambda a, b, s: [ai + s * bi if ai is not None else None for ai, bi in zip(a, b)]
    # predictor: RK4 from node to node
    Y, cur, t = [], y, 0.0
    for cm in c:
        h = (cm - t) * dt
        k1 = F(cur)
        k2 = F(add(cur, k1, h / 2))
        k3 = F(add(cur, k2, h / 2))
        k4 = F(add(cur, k3, h))
        cur = add(add(add(add(cur, k1, h / 6), k2, h / 3), k3, h / 3), k4, h / 6)
        Y.append(cur)
        t = cm
    # correction sweeps, then the final integration
    for _ in range(sweeps):
        FY = [F(Ym) for Ym in Y]
        newY = []
        for m in range(len(c)):
            acc = list(y)
            for j in range(len(c)):
                acc = add(acc, FY[j], dt * S[m][j])
            newY.append(acc)
        Y = newY
    FY = [F(Ym) for Ym in Y]
    out = list(y)
    for j in range(len(c)):
        out = add(out, FY[j], dt * S[-1][j])
    return out


def march_sdc(eta0, phi0, Qe0, Qp0, h, tau, g, T, nsteps, sweeps=SWEEPS, ar=O.F64):
    """nsteps SDC15 steps of dt = T / (4 nsteps) for (q, Qdot), the filter applied to the
    state after every step.  ar: one of ww_oracle's FP64 backends (the right-hand sides
    and the filter run in it; the step's combinations are plain FP64)."""
    c = radau_iia_nodes()
    S = integration_matrix(c)
    dt = T / (4 * nsteps)
    F = lambda y: list(O.rhs(y[0], y[1], y[2], y[3], h, tau, g, ar))
    y = [eta0, phi0, Qe0, Qp0]
    for _ in range(nsteps):
        y = sdc_step(y, F, dt, c, S, sweeps)
        y = [O.filt(v, ar) if v is not None else None for v in y]
    return y


def shoot_eval_sdc(N, h, tau, g, basis, q_fixed, params, T, nsteps, jacobian=True, sweeps=SWEEPS, ar=O.F64):
    """r, J, dr/dT, f as oracle.ww_oracle.shoot_eval, marched with SDC15 (ar: as for
    march_sdc)."""
    basis = np.asarray(basis, dtype=float)
    q0 = np.asarray(q_fixed, dtype=float) + ar.matmul(basis, np.asarray(params, dtype=float))
    Qe, Qp = (basis[:N], basis[N:]) if jacobian else (None, None)
    eta, phi, Qe, Qp = march_sdc(q0[:N], q0[N:], Qe, Qp, h, tau, g, T, nsteps, sweeps, ar)
    w = 1 / math.sqrt(N)
    _, phi_t, _, _ = O.rhs(eta, phi, None, None, h, tau, g, ar)
    r = w * phi
    return dict(r=r, J=(w * Qp) if jacobian else None, drdT=w * phi_t / 4, f=math.fsum(r * r) / 2,
                eta=eta, phi=phi)


def shoot_eval_sdc_dd(N, h, tau, g, eta0, phi0, T, nsteps, sweeps=SWEEPS):
    """The base march (no Jacobian) in double-double with SDC15 (the paper's quadruple-
    precision workflow, Sec. 2.2): eta0, phi0 and T double-doubles (oracle.dd.DD), the
    right-hand sides, filter and step in double-double, the nodes and weights to about
    32 digits.  Returns r, dr/dT, f (double-double) as shoot_eval_sdc."""
    from . import dd as D
    ar = D.DDArith()
    c, S = nodes_and_matrix_dd()
    T = D._dd(T)
    dt = T / (4 * nsteps)
    F = lambda y: list(O.rhs(y[0], y[1], None, None, h, tau, g, ar))[:2] + [None, None]
    y = [D._dd(eta0), D._dd(phi0), None, None]
    for _ in range(nsteps):
        y = sdc_step(y, F, dt, c, S, sweeps)
        y = [O.filt(v, ar) if v is not None else None for v in y]
    eta, phi = y[0], y[1]
    w = 1 / D.sqrt(D.DD(float(N)))
    _, phi_t, _, _ = O.rhs(eta, phi, None, None, h, tau, g, ar)
    r = w * phi
    return dict(r=r, drdT=w * phi_t / 4, f=D.dd_sum(r * r) / 2, eta=eta, phi=phi)
