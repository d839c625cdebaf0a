"""BFGS with a strong-Wolfe line search: the adjoint-continuation (ACM) minimiser of
Sec. 3.2 -- test infrastructure.

The oracle of the GPU driver `ww_bfgs`: NumPy, used only by the tests.  The paper names
the method (BFGS, a quasi-Newton method building an inverse-Hessian approximation from
the gradients met on successive line searches) but not its parameters; the readings:
  B1  inverse-Hessian form of the BFGS update, H_{k+1} = (I - rho s y^T) H_k (I - rho y s^T)
      + rho s s^T, rho = 1 / y^T s, skipped when y^T s <= 0; before the first update
      H_0 = I, replaced once by (s^T y / y^T y) I before the first update is applied.
  B2  strong Wolfe conditions with c1 = 1e-4, c2 = 0.9; the first trial step of each line
      search is 1, capped by a step length of delta0 / ||p|| on the first iteration;
      bracketing by doubling (at most 20 times), zoom by bisection (at most 30 times);
      a line search that ends without the conditions takes the best point found if it
      decreases f, else the run stops.
  B3  stop when f < f_tol, ||g|| < g_tol, the step leaves c unchanged, or after
      max_iter iterations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

C1, C2 = 1e-4, 0.9


@dataclass
class BfgsResult:
    c: np.ndarray
    f: float
    g: np.ndarray
    reason: str
    evals: int
    history: list = field(default_factory=list)   # (c, f) after every iteration


def line_search(fg, c, f0, g0, p, a1):
    """Strong-Wolfe search along p from c (directional derivative g0.p < 0).
    Returns (alpha, f, g, evals, ok)."""
    d0 = float(g0 @ p)
    evals = 0
    a_prev, f_prev = 0.0, f0
    a = a1
    best = (0.0, f0, g0)
    lo = hi = None
    for i in range(20):
        f, g = fg(c + a * p)
        evals += 1
        if f < best[1]:
            best = (a, f, g)
        if f > f0 + C1 * a * d0 or (i > 0 and f >= f_prev):
            lo, flo, hi = a_prev, f_prev, a
            break
        d = float(g @ p)
        if abs(d) <= -C2 * d0:
            return a, f, g, evals, True
        if d >= 0:
            lo, flo, hi = a, f, a_prev
            break
        a_prev, f_prev = a, f
        a = 2.0 * a
    else:
        return best[0], best[1], best[2], evals, False
    for _ in range(30):   # zoom by bisection between lo (sufficient decrease) and hi
        a = 0.5 * (lo + hi)
        f, g = fg(c + a * p)
        evals += 1
        if f < best[1]:
            best = (a, f, g)
        if f > f0 + C1 * a * d0 or f >= flo:
            hi = a
        else:
            d = float(g @ p)
            if abs(d) <= -C2 * d0:
                return a, f, g, evals, True
            if d * (hi - lo) >= 0:
                hi = lo
            lo, flo = a, f
    return best[0], best[1], best[2], evals, False


def bfgs(fg, c0, delta0=0.1, f_tol=1e-26, g_tol=1e-13, max_iter=200):
    """fg(c) -> (f, g).  Returns BfgsResult; reasons "f_tol", "g_tol", "c unchanged",
    "line search", "max_iter"."""
    c = np.array(c0, dtype=np.float64)
    f, g = fg(c)
    evals = 1
    n = c.size
    H = np.eye(n)
    first = True
    hist = []
    for it in range(max_iter):
        if f < f_tol:
            return BfgsResult(c, f, g, "f_tol", evals, hist)
        if np.linalg.norm(g) < g_tol:
            return BfgsResult(c, f, g, "g_tol", evals, hist)
        p = -H @ g
        if float(g @ p) >= 0:   # not a descent direction: restart from steepest descent
            H = np.eye(n)
            p = -g
        a1 = min(1.0, delta0 / np.linalg.norm(p)) if first else 1.0
        a, fn, gn, ne, ok = line_search(fg, c, f, g, p, a1)
        evals += ne
        if not ok and not fn < f:
            return BfgsResult(c, f, g, "line search", evals, hist)
        cn = c + a * p
        if np.array_equal(cn, c):
            return BfgsResult(c, f, g, "c unchanged", evals, hist)
        s, y = cn - c, gn - g
        sy = float(s @ y)
        if sy > 0:
            if first:
                H = (sy / float(y @ y)) * np.eye(n)
            rho = 1.0 / sy
            V = np.eye(n) - rho * np.outer(y, s)
            H = V.T @ H @ V + rho * np.outer(s, s)
            first = False
        c, f, g = cn, fn, gn
        hist.append((c.copy(), f))
    return BfgsResult(c, f, g, "max_iter", evals, hist)
