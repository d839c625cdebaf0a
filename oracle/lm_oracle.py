"""Levenberg-Marquardt with delayed Jacobian updates (App. C) -- test infrastructure.

This module is the oracle of the trust-region driver that is built on the shooting
evaluation: a plain NumPy statement of App. C, used only by the tests and by nothing on
the GPU path.  It minimises f(c) = r(c).r(c)/2 for a residual function r and its
Jacobian J (App. C, first display), solving each trust-region subproblem through the
thin SVD of J (App. C, eq. (trust:tilde)) with a Newton iteration on
tau(lambda) = 1/||p~|| - 1/Delta, and re-using J over several steps by the rules 1-4 of
App. C.

Readings (the appendix is silent or garbled here):
  L1  The printed Newton update for lambda divides by p~^T (S^T S + lambda I) p~; the
      Newton step of tau(lambda) for p~_k = -sigma_k r~_k / (sigma_k^2 + lambda) divides
      by p~^T (S^T S + lambda I)^{-1} p~ (the units of lambda are those of sigma^2), so
      the inverse is read as intended.
  L2  delta_first_rejected is set once per Jacobian: the first radius rejected
      (rho < rho_0) at or after the first accepted step since J was computed; it is
      cleared when J is recomputed.
  L3  Rule 3's test |df|/f < df_tol uses the df of the step just tried and the f of the
      current iterate after that step.
  L4  Singular values below n eps sigma_max count as zero (the minimum-norm solution of
      the subproblem).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# App. C, rules 1-3
F_TOL = 1e-26
G_TOL = 1e-13
DF_TOL = 1e-5
MAX_STEPS_J = 10
RHO0, RHO1 = 0.25, 0.85
ALPHA0, ALPHA1, ALPHA2 = 3.0 / 8.0, 1.875, 0.2
NEWTON_TOL = 1e-12


def tilde_step(sigma, rt, lam):
    """p~(lambda) = argmin ||[S; sqrt(lambda) I] p~ + [r~; 0]||, componentwise
    -sigma_k r~_k / (sigma_k^2 + lambda) (zero for sigma_k = 0)."""
    den = sigma * sigma + lam
    out = np.zeros_like(rt)
    nz = sigma > 0
    out[nz] = -sigma[nz] * rt[nz] / den[nz]
    return out


def trust_subproblem(sigma, rt, delta, tol=NEWTON_TOL, maxit=200):
    """Solve eq. (trust:tilde): returns (p~, lambda).  lambda = 0 when the unconstrained
    minimum-norm step lies inside the region (tau(0) >= 0); otherwise the Newton
    iteration on tau from lambda = 0 (reading L1) increases monotonically to the root."""
    p = tilde_step(sigma, rt, 0.0)
    if np.linalg.norm(p) <= delta:
        return p, 0.0
    lam = 0.0
    for _ in range(maxit):
        pn = np.linalg.norm(p)
        if abs(pn - delta) / delta <= tol:
            break
        nz = sigma > 0
        q = np.sum(p[nz] * p[nz] / (sigma[nz] ** 2 + lam))   # p~^T (S^T S + lambda I)^{-1} p~
        lam = lam + (pn * pn / q) * ((pn - delta) / delta)
        p = tilde_step(sigma, rt, lam)
    return p, lam


def thin_svd(J):
    """J = U S V^T (thin) with small singular values zeroed (reading L4)."""
    U, s, Vt = np.linalg.svd(J, full_matrices=False)
    if s.size and s[0] > 0:
        s = np.where(s < s.size * np.finfo(float).eps * s[0], 0.0, s)
    return U, s, Vt.T


@dataclass
class LMResult:
    c: np.ndarray
    f: float
    reason: str
    evals_r: int
    evals_J: int
    history: list = field(default_factory=list)   # (c, f, accepted, delta) per tried step


def levmar(residual, jacobian, c0, delta0, f_tol=F_TOL, g_tol=G_TOL, df_tol=DF_TOL,
           max_steps_J=MAX_STEPS_J, max_evals=200):
    """App. C.  residual(c) -> r; jacobian(c) -> (r, J).  Returns LMResult.

    Reasons: "f=0", "c unchanged", "roundoff: rejected", "roundoff: max_stepsJ",
    "max_evals"."""
    c = np.array(c0, dtype=np.float64)
    r, J = jacobian(c)
    evals_r, evals_J = 0, 1
    f = 0.5 * float(r @ r)
    U, s, V = thin_svd(J)
    steps_J = 0
    delta = float(delta0)
    roundoff = False
    dfr = None               # delta_first_rejected of this Jacobian (reading L2)
    accepted_since_J = False
    hist = []
    while True:
        if f == 0.0:
            return LMResult(c, f, "f=0", evals_r, evals_J, hist)
        if evals_r + evals_J >= max_evals:
            return LMResult(c, f, "max_evals", evals_r, evals_J, hist)
        rt = U.T @ r
        pt, _ = trust_subproblem(s, rt, delta)
        p = V @ pt
        # predicted change of the quadratic model: g.p + p.B.p/2 in the SVD basis
        df = float((s * rt) @ pt + 0.5 * np.sum((s * pt) ** 2))
        g = V @ (s * rt)
        if f < f_tol or delta < g_tol:
            roundoff = True
        if steps_J == 0 and (np.linalg.norm(g) < g_tol or abs(df) / f < df_tol):
            roundoff = True
        cn = c + p
        if np.array_equal(cn, c):
            return LMResult(c, f, "c unchanged", evals_r, evals_J, hist)
        rn = residual(cn)
        evals_r += 1
        fn = 0.5 * float(rn @ rn)
        rho = (fn - f) / df if df != 0.0 else -1.0
        accepted = rho > 0.0
        pnorm = float(np.linalg.norm(p))
        hist.append((cn.copy(), fn, accepted, delta))
        if accepted:
            accepted_since_J = True
        if rho < RHO0:
            if dfr is None and accepted_since_J:
                dfr = delta
            delta = ALPHA0 * pnorm
        elif rho > RHO1 and pnorm > 0.9 * delta:
            delta = ALPHA1 * delta
        if accepted:
            c, r, f = cn, rn, fn
            steps_J += 1
        if roundoff and (not accepted or steps_J >= max_steps_J):
            return LMResult(c, f, "roundoff: rejected" if not accepted else "roundoff: max_stepsJ",
                            evals_r, evals_J, hist)
        trigger = ALPHA2 * dfr if dfr is not None else -math.inf
        if not roundoff and (steps_J >= max_steps_J or (steps_J > 0 and delta < trigger)
                             or (steps_J > 0 and f > 0 and abs(df) / f < df_tol)):
            if dfr is not None:
                delta = dfr / ALPHA1
            r, J = jacobian(c)
            evals_J += 1
            f = 0.5 * float(r @ r)
            U, s, V = thin_svd(J)
            steps_J = 0
            dfr = None
            accepted_since_J = False
