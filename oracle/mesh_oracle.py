"""CPU reference ("oracle") for the non-uniform mesh with time segments of Wilkening &
Yu (Sec. 2.2 eq. (xi), (rho:def)): the DtN operator, the right-hand sides and the
DOP853 (or SDC15) march on the mapped grid x = xi(alpha), and the regridding between time
segments.

TEST INFRASTRUCTURE ONLY, like oracle/ww_oracle.py (whose spectral operators, cot
branch formula, tableau and FP64 arithmetic backends it uses); it shares no code with
the GPU library.  FP64 numpy backends only (the default and the alternate roundings).

What is computed (N points alpha_j = 2 pi j / N on segment l, the state eta, varphi
and the Jacobian columns held at x_j = xi(alpha_j)):

  * Sec. 2.2 eq. (xi): E = xi' = 1 - P[A sin^4(alpha/2)] (refine near x = pi) or
    1 - P[A cos^4(alpha/2)] (refine near x = 0), A = 8 (1 - rho) / (5 + 3 rho); P
    removes the mean (3/8), and xi = int_0^alpha E in closed form.
  * Sec. 2.1 eq. (zeta): zeta = xi + i eta, so zeta' = E + i eta_alpha and
    zeta'' = E' + i eta_alphaalpha (alpha-derivatives spectral, on the uniform grid).
  * Sec. 2.2 / App. A: eq. (fred) by trapezoidal collocation in alpha with the (K1K2)
    kernels of the general curve (the subtracted cot((alpha - beta)/2)/2 stays in
    alpha); eq. (G): G varphi = [H gamma / 2 + int G gamma] / |xi'|.
  * Sec. 2.1 eq. (ww), (uv:from:G) and App. B (l4)-(l6a) with d/dx = (1/E) d/dalpha.
  * Time segments theta_l T, each with its own N_l, step count and rho_l; between
    segments the state and every Jacobian column are carried to the new mesh by
    evaluating the trigonometric interpolant (in alpha) of the old values at
    beta_j = xi_l^{-1}(xi_{l+1}(alpha_j)) (the regridding described with eq. (xi)).

Readings (listed with the design notes):
  M1  P in eq. (ww:2) is the zero-mean projection in x: on the mapped grid the mean is
      the E-weighted trapezoidal sum, P f = f - (1/N) sum_j E_j f_j.
  M2  the filter (filter) acts on the Fourier coefficients in alpha (the uniform grid
      of the discretisation), as on the uniform mesh.
  M3  the objective weights of eq. (f:phi) are r_i = varphi_i sqrt(E_i / N) on the
      last segment's mesh (R10 with the mesh spacing), and J, dr/dT carry the same
      weights; dr/dT = (1/4) w varphi_t at T/4 (R5: the segments' step sizes all
      scale with T).
  M4  the interpolant of the regridding is the trigonometric one of degree N/2 with
      the Nyquist mode as a cosine (real, reproduces the values at the grid points).
  M5  the mesh safety rule is enforced: if rho_{l+1} < rho_l then
      N_{l+1} / N_l >= (5 + 3 rho_l) / (5 + 3 rho_{l+1}).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.optimize

from . import ww_oracle as O

REFINE_PI, REFINE_ZERO = 0, 1


class Mesh:
    """The change of variables x = xi(alpha) of Sec. 2.2 eq. (xi) on N points."""

    def __init__(self, N: int, rho: float = 1.0, refine_at: int = REFINE_PI):
        if not (0.0 < rho <= 1.0):
            raise ValueError("rho must lie in (0, 1]")
        if refine_at not in (REFINE_PI, REFINE_ZERO):
            raise ValueError("refine_at must be REFINE_PI or REFINE_ZERO")
        self.N, self.rho, self.refine_at = N, float(rho), refine_at
        self.A = 8.0 * (1.0 - rho) / (5.0 + 3.0 * rho)
        alpha = 2.0 * np.pi * np.arange(N) / N
        self.alpha = alpha
        self.xi = self.xi_at(alpha)
        self.E = self.E_at(alpha)
        self.Ep = self.Ep_at(alpha)

    # sin^4(a/2) = (3 - 4 cos a + cos 2a)/8, cos^4(a/2) = (3 + 4 cos a + cos 2a)/8:
    # the projected profile, its derivative and its integral from 0
    def _sgn(self):
        return -1.0 if self.refine_at == REFINE_PI else 1.0

    def E_at(self, a):
        a = np.asarray(a, dtype=float)
        prof = (self._sgn() * 4.0 * np.cos(a) + np.cos(2.0 * a)) / 8.0    # s - 3/8
        return 1.0 - self.A * prof

    def Ep_at(self, a):
        a = np.asarray(a, dtype=float)
        dprof = (-self._sgn() * 4.0 * np.sin(a) - 2.0 * np.sin(2.0 * a)) / 8.0
        return -self.A * dprof

    def xi_at(self, a):
        a = np.asarray(a, dtype=float)
        iprof = (self._sgn() * 4.0 * np.sin(a) + 0.5 * np.sin(2.0 * a)) / 8.0
        return a - self.A * iprof

    def xi_inverse(self, x):
        """alpha with xi(alpha) = x: bracketed root finding (xi is increasing and
        |xi(a) - a| <= 9 A / 16 < 1), then two Newton steps to the rounding level."""
        out = np.empty(len(x))
        for j, xj in enumerate(np.asarray(x, dtype=float)):
            b = scipy.optimize.brentq(lambda t: float(self.xi_at(t)) - xj, xj - 1.0, xj + 1.0,
                                      xtol=1e-15, rtol=1e-15, maxiter=200)
            for _ in range(2):
                b -= (float(self.xi_at(b)) - xj) / float(self.E_at(b))
            out[j] = b
        return out


def check_segments(segments):
    """Validate a list of segments (dicts with N, nsteps, theta, rho, refine_at)."""
    if not segments:
        raise ValueError("at least one segment")
    if abs(math.fsum(s["theta"] for s in segments) - 1.0) > 1e-12:
        raise ValueError("the segment fractions theta must sum to 1")
    for a, b in zip(segments[:-1], segments[1:]):
        if b["rho"] < a["rho"] and b["N"] * (5.0 + 3.0 * b["rho"]) < a["N"] * (5.0 + 3.0 * a["rho"]) * (1 - 1e-15):
            raise ValueError("refining the mesh needs N_{l+1}/N_l >= (5 + 3 rho_l)/(5 + 3 rho_{l+1})")


# --------------------------------------------------------------------------------
# DtN on the mapped grid, Sec. 2.1-2.2 and App. A
# --------------------------------------------------------------------------------

def assemble_mapped(eta, h, mesh: Mesh, ar=O.F64):
    """A = I/2 + K/N and Gm = G/N of eq. (fred) and (G) for the curve
    zeta = xi + i eta, with the (K1K2) kernels (reading R1 for the image terms)."""
    N = eta.shape[0]
    E, Ep, xi, alpha = mesh.E, mesh.Ep, mesh.xi, mesh.alpha
    et = O.surface_height(eta, h)
    ex = O.deriv(eta, ar)           # Im zeta'  (alpha-derivative)
    exx = O.deriv(ex, ar)           # Im zeta''
    x = xi[:, None] - xi[None, :]
    y = et[:, None] - et[None, :]
    xo = x.copy()
    ao = alpha[:, None] - alpha[None, :]
    for i in range(N):
        xo[i, i] = np.pi
        ao[i, i] = np.pi
    cre, cim = O.cot_half(xo, y, ar)
    c0re, _ = O.cot_half(ao, 0 * ao, ar)
    c0 = c0re / 2
    # K1 = Im{zeta'_j C}/2 with zeta'_j = E_j + i ex_j; G1 = Re{zeta'_i C}/2 - c0
    K = (E[None, :] * cim + ex[None, :] * cre) / 2
    G = (E[:, None] * cre - ex[:, None] * cim) / 2 - c0
    # diagonal: zeta''/zeta' = (Ep + i exx)(E - i ex) / (E^2 + ex^2)
    den = E * E + ex * ex
    kd = -((exx * E - Ep * ex) / den) / 2
    gd = ((Ep * E + exx * ex) / den) / 2
    for i in range(N):
        K[i, i] = kd[i]
        G[i, i] = gd[i]
    if not math.isinf(h):
        yb = et[:, None] + et[None, :]
        dre, dim = O.cot_half(x, yb, ar)
        # K2 = -Im{conj(zeta'_j) D}/2, G2 = -Re{zeta'_i D}/2
        K = K - (E[None, :] * dim - ex[None, :] * dre) / 2
        G = G - (E[:, None] * dre - ex[:, None] * dim) / 2
    A = K / N + np.eye(N) / 2
    return A, G / N


class DtNMapped:
    """Assemble, factor once, apply to any number of right-hand sides."""

    def __init__(self, eta, h, mesh: Mesh, ar=O.F64):
        self.mesh, self.ar = mesh, ar
        self.A, self.Gm = assemble_mapped(eta, h, mesh, ar)
        self.lu = ar.lu_factor(self.A)

    def apply(self, psi):
        """G psi = [H gamma / 2 + Gm gamma] / E, gamma = d mu / d alpha, A mu = psi."""
        ar = self.ar
        mu = ar.lu_solve(self.lu, psi)
        gam = O.deriv(mu, ar)
        out = O.hilbert(gam, ar) / 2 + ar.matmul(self.Gm, gam)
        E = self.mesh.E
        return (out / E[:, None] if out.ndim == 2 else out / E), mu


def _dx(f, E, ar=O.F64):
    """d/dx = (1/E) d/dalpha."""
    d = O.deriv(f, ar)
    return d / E[:, None] if d.ndim == 2 else d / E


def _proj_x(f, E):
    """Reading M1: zero mean in x, the E-weighted trapezoidal mean."""
    N = f.shape[0]
    if f.ndim == 2:
        return f - (E @ f)[None, :] / N
    return f - np.dot(E, f) / N


def rhs_mapped(eta, phi, Qe, Qp, h, tau, g, mesh: Mesh, ar=O.F64):
    """F(q) and DF(q) Qdot on the mapped grid (eq. (ww), App. B), filtered (R7, M2)."""
    E = mesh.E
    dtn = DtNMapped(eta, h, mesh, ar)
    ex = _dx(eta, E, ar)
    ps = _dx(phi, E, ar)
    Gphi, _ = dtn.apply(phi)
    den = 1 + ex * ex
    u = (ps - ex * Gphi) / den
    v = (ex * ps + Gphi) / den
    curv = _dx(ex / np.sqrt(den), E, ar)
    phi_t = _proj_x(v * Gphi - u * u / 2 - v * v / 2 - g * eta + tau * curv, E)
    eta_t = O.filt(Gphi, ar)
    phi_t = O.filt(phi_t, ar)
    if Qe is None:
        return eta_t, phi_t, None, None
    psid = Qp - v[:, None] * Qe                                    # (l4)
    Gpsid, _ = dtn.apply(psid)
    Qe_t = Gpsid - _dx(Qe * u[:, None], E, ar)                     # (l5a)
    dpsid = _dx(psid, E, ar)
    w3 = den * np.sqrt(den)
    tens = _dx(_dx(Qe, E, ar) / w3[:, None], E, ar)
    Qp_t = _proj_x(-_dx(Qe * (u * v)[:, None], E, ar) - u[:, None] * dpsid
                   + v[:, None] * Gpsid - g * Qe + tau * tens, E)  # (l6), (l6a)
    return eta_t, phi_t, O.filt(Qe_t, ar), O.filt(Qp_t, ar)


def march_mapped(eta0, phi0, Qe0, Qp0, h, tau, g, T, nsteps, mesh: Mesh, tableau=None, ar=O.F64):
    """nsteps fixed DOP853 steps of dt = T / (4 nsteps) on one mesh (T here is the
    simulated span times 4, as in oracle.ww_oracle.march)."""
    a, b, c = tableau if tableau is not None else O.dop853_tableau()
    s = len(b)
    dt = T / (4 * nsteps)
    y = [eta0, phi0, Qe0, Qp0]
    for _ in range(nsteps):
        ks = []
        for i in range(s):
            Y = list(y)
            for j in range(i):
                if a[i, j] != 0.0:
                    Y = [Y[q] + a[i, j] * dt * ks[j][q] if Y[q] is not None else None for q in range(4)]
            ks.append(rhs_mapped(Y[0], Y[1], Y[2], Y[3], h, tau, g, mesh, ar))
        yn = list(y)
        for i in range(s):
            if b[i] != 0.0:
                yn = [yn[q] + b[i] * dt * ks[i][q] if yn[q] is not None else None for q in range(4)]
        y = [O.filt(v, ar) if v is not None else None for v in yn]
    return y


def march_mapped_sdc(eta0, phi0, Qe0, Qp0, h, tau, g, T, nsteps, mesh: Mesh, ar=O.F64):
    """nsteps SDC15 steps of dt = T / (4 nsteps) on one mesh: the step of
    oracle/sdc_oracle.py with the mapped right-hand sides, the filter after every step."""
    from . import sdc_oracle as S
    c = S.radau_iia_nodes()
    Sm = S.integration_matrix(c)
    dt = T / (4 * nsteps)
    F = lambda y: list(rhs_mapped(y[0], y[1], y[2], y[3], h, tau, g, mesh, ar))
    y = [eta0, phi0, Qe0, Qp0]
    for _ in range(nsteps):
        y = S.sdc_step(y, F, dt, c, Sm)
        y = [O.filt(v, ar) if v is not None else None for v in y]
    return y


# --------------------------------------------------------------------------------
# regridding between segments
# --------------------------------------------------------------------------------

def trig_interp(values, beta):
    """Trigonometric interpolant (reading M4) of values on the uniform alpha grid of
    N = len(values) points, evaluated at the points beta; columns independent."""
    v = np.asarray(values, dtype=float)
    N = v.shape[0]
    F = np.fft.rfft(v, axis=0) / N
    k = np.arange(N // 2 + 1)
    wk = np.full(N // 2 + 1, 2.0)
    wk[0] = 1.0
    wk[N // 2] = 1.0                         # the Nyquist mode as a cosine
    ph = np.exp(1j * np.outer(beta, k))      # (len(beta), N/2 + 1)
    return ((ph * wk[None, :]) @ F).real


def regrid(values, old: Mesh, new: Mesh):
    """Values at x = xi_old(alpha_j) carried to x = xi_new(alpha_j) of the new grid."""
    beta = old.xi_inverse(new.xi)
    return trig_interp(values, beta)


# --------------------------------------------------------------------------------
# the segmented march and its outputs
# --------------------------------------------------------------------------------

def shoot_eval_segments(N, h, tau, g, basis, q_fixed, params, T, segments, jacobian=True, tableau=None,
                        ar=O.F64, scheme="dop853"):
    """r, J, dr/dT, f after marching the segments to T/4 (readings M1-M5).

    segments: dicts with N (segments[0]["N"] == N), nsteps, theta, rho, refine_at.
    basis (2N, M) and q_fixed (2N,) are values on the first segment's mesh.  `ar`: one of
    the FP64 backends of ww_oracle (the alternates round the same scheme differently,
    to measure the rounding floor).  scheme: "dop853" or "sdc" (SDC15 steps, Sec. 2.2)."""
    if scheme not in ("dop853", "sdc"):
        raise ValueError(scheme)
    check_segments(segments)
    if segments[0]["N"] != N:
        raise ValueError("the basis lives on the first segment's grid")
    basis = np.asarray(basis, dtype=float)
    q0 = np.asarray(q_fixed, dtype=float) + basis @ np.asarray(params, dtype=float)
    eta, phi = q0[:N], q0[N:]
    Qe, Qp = (basis[:N], basis[N:]) if jacobian else (None, None)
    mesh = None
    for seg in segments:
        new = Mesh(seg["N"], seg["rho"], seg.get("refine_at", REFINE_PI))
        if mesh is not None:
            eta, phi = regrid(eta, mesh, new), regrid(phi, mesh, new)
            if jacobian:
                Qe, Qp = regrid(Qe, mesh, new), regrid(Qp, mesh, new)
        mesh = new
        if scheme == "sdc":
            eta, phi, Qe, Qp = march_mapped_sdc(eta, phi, Qe, Qp, h, tau, g, seg["theta"] * T, seg["nsteps"], mesh, ar)
        else:
            eta, phi, Qe, Qp = march_mapped(eta, phi, Qe, Qp, h, tau, g, seg["theta"] * T, seg["nsteps"], mesh,
                                            tableau, ar)
    w = np.sqrt(mesh.E / mesh.N)
    r = w * phi
    _, phi_t, _, _ = rhs_mapped(eta, phi, None, None, h, tau, g, mesh, ar)
    return dict(r=r, J=(w[:, None] * Qp) if jacobian else None, drdT=w * phi_t / 4,
                f=math.fsum(r * r) / 2, eta=eta, phi=phi, mesh=mesh)


def energy_mapped(eta, phi, h, tau, g, mesh: Mesh):
    """E = int [phi G phi / 2 + g eta^2 / 2 + tau (sqrt(1 + eta_x^2) - 1)] dx on the
    mapped grid, (2 pi / N) sum_j E_j (...)_j (R12 with the mesh spacing)."""
    Gphi, _ = DtNMapped(eta, h, mesh).apply(phi)
    ex = _dx(eta, mesh.E)
    e = phi * Gphi / 2 + g * eta * eta / 2 + tau * (np.sqrt(1 + ex * ex) - 1)
    return 2 * np.pi / mesh.N * math.fsum(mesh.E * e)
