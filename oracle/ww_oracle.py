"""CPU reference ("oracle") for the Dirichlet-Neumann / Jacobian hot path of
Wilkening & Yu, "Overdetermined shooting methods for computing standing water
waves with spectral accuracy".

TEST INFRASTRUCTURE ONLY.  This module is imported by tests/, by the smoke check
and by the CPU-baseline timing of the benchmark.  The product path never imports
it, and it shares no code with the GPU library: the only module both sides use is
the seeded input generator.

Plain, slow, obviously correct: FP64 numpy, with numpy.fft for Fourier
multipliers and scipy's partially pivoted LU for the dense solve.  The same code
also runs in extended precision (mpmath, see oracle/xprec.py) through the small
arithmetic backend `Arith` below, to measure the FP64 rounding floor.

What is computed, in the paper's order and notation (N grid points, alpha_j =
2 pi j / N, uniform mesh xi(alpha) = alpha, so E = 1 and |xi'| = 1):

  * Sec. 2.1 eq. (ww): eta_t = phi_y - eta_x phi_x,
    varphi_t = P[phi_y eta_t - u^2/2 - v^2/2 - g eta + tau d/dx(eta_x / sqrt(1+eta_x^2))],
    with (u, v) = (phi_x, phi_y) from eq. (uv:from:G).
  * Sec. 2.2 / App. A: second-kind Fredholm equation (fred) solved by trapezoidal
    collocation, kernels (K1K2) with the cot branch formula of Sec. 2.2, regularised
    diagonals, the DtN formula (G) / (DNO:formula) with gamma = mu'.
  * Sec. 2.2: 36th-order filter (filter) on the right-hand side at every stage and on
    the solution after every step; DOP853 (12 stages for the 8th-order update).
  * Sec. 3.3 eq. (q:qdot): base state and the Jacobian columns evolved together with
    one DtN (one LU) per stage; the variational right-hand side is App. B eq. (l5a),
    (l6), (l6a).
  * Sec. 3.1 eq. (f:phi) and Sec. 3.3 eq. (Jik): r, J, f; Sec. 3.2 eq. (dfdT) for the
    T-derivative.

Readings where the paper is silent, garbled or inconsistent (each is listed with
the design notes):
  R1  image terms enter with a minus sign: K2 = -Im{conj(zeta'(beta))/2 cot((zeta(alpha)-conj zeta(beta))/2)},
      G2 = -Re{zeta'(alpha)/2 cot(...)}, as the bracket of eq. (Phi) and (plemelj:1/2)
      gives (the printed (K1K2) shows "+").
  R2  the subtracted (1/2)cot((alpha-beta)/2) is real and drops out of K1 = Im{...}.
  R3  `eta` is the displacement; at finite depth h the surface height is h + eta
      (bottom at y = 0, App. A); the gravity term uses the displacement (P removes
      the constant g h exactly in exact arithmetic).
  R5  drdT = (1/4) w phi_t(T/4): T is the full period and the march ends at T/4.
  R6  d/dx and H zero the Nyquist mode; the filter multiplies it by exp(-36).
  R7  the filter is applied to both right-hand sides and to every Jacobian column.
  R8  DOP853 with the 12-stage 8th-order update, fixed steps, no FSAL reuse.
  R9  the gradient is J^T r of the discretised variational scheme.
  R10 r = phi(T/4) / sqrt(N), f = r.r / 2.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

# --------------------------------------------------------------------------------
# arithmetic backend (FP64 numpy).  oracle/xprec.py provides the same interface on
# mpmath objects.
# --------------------------------------------------------------------------------


def _kvec(N: int) -> np.ndarray:
    """Wavenumbers of numpy's real FFT, k = 0..N/2."""
    return np.arange(N // 2 + 1, dtype=float)


def multiplier(kind: str, N: int, k: np.ndarray) -> np.ndarray:
    """Fourier symbols on k = 0..N/2 (real-FFT half spectrum), Sec. 2.2 and App. A.

    'd' : d/dx -> i k, Nyquist set to zero (reading R6)
    'h' : Hilbert transform -> -i sgn(k), zero at k = 0 and at Nyquist
    'p' : P, projection to zero mean -> zero at k = 0
    'f' : filter (filter): exp(-36 (|k| / (N/2))^36), Nyquist included
    """
    nyq = N // 2
    m = np.zeros(k.shape, dtype=complex)
    if kind == "d":
        m = 1j * k
        m[k == nyq] = 0.0
    elif kind == "h":
        m = -1j * np.sign(k)
        m[k == nyq] = 0.0
    elif kind == "p":
        m = np.ones(k.shape, dtype=complex)
        m[k == 0] = 0.0
    elif kind == "f":
        m = np.exp(-36.0 * (k / nyq) ** 36).astype(complex)
    else:
        raise ValueError(kind)
    return m


class Arith:
    """FP64 backend: numpy arrays, numpy.fft, scipy LU with partial pivoting."""

    name = "f64"

    def __init__(self):
        self._mult = {}

    # scalars / elementwise
    def const(self, x):
        return float(x)

    def asarray(self, x):
        return np.array(x, dtype=float)

    def zeros(self, shape):
        return np.zeros(shape)

    def grid(self, N):
        """Collocation points alpha_j = 2 pi j / N."""
        return 2.0 * np.pi * np.arange(N) / N

    sin = staticmethod(np.sin)
    cos = staticmethod(np.cos)
    exp = staticmethod(np.exp)
    sqrt = staticmethod(np.sqrt)

    @property
    def pi(self):
        return np.pi

    def spectral(self, kind: str, f):
        """Apply a Fourier multiplier along axis 0 (columns are independent)."""
        N = f.shape[0]
        key = (kind, N)
        if key not in self._mult:
            self._mult[key] = multiplier(kind, N, _kvec(N))
        m = self._mult[key]
        fh = np.fft.rfft(f, axis=0)
        if f.ndim == 2:
            fh = fh * m[:, None]
        else:
            fh = fh * m
        return np.fft.irfft(fh, n=N, axis=0)

    def lu_factor(self, A):
        return scipy.linalg.lu_factor(A)

    def lu_solve(self, lu, B):
        return scipy.linalg.lu_solve(lu, B)

    def matmul(self, A, B):
        return A @ B

    def sum(self, x):
        return math.fsum(np.ravel(x))

    def where(self, c, a, b):
        return np.where(c, a, b)

    def ge0(self, x):
        return x >= 0.0

    def cosh_sinh(self, y):
        """cosh y, sinh y from exp(y) and exp(-y)."""
        ey = np.exp(y)
        eyi = np.exp(-y)
        return (ey + eyi) / 2, (ey - eyi) / 2


class ArithAlt(Arith):
    """The same FP64 arithmetic with cosh and sinh taken from the math library: a
    second, equally valid rounding of the same formulas.  Used only to measure the
    FP64 rounding floor of long marches (the spread between the two runs)."""

    name = "f64alt"

    def cosh_sinh(self, y):
        return np.cosh(y), np.sinh(y)


class ArithAltFFT(Arith):
    """The same FP64 arithmetic with every Fourier multiplier applied through the full
    complex FFT (numpy.fft.fft / ifft) instead of the real-input transforms: the same
    operator, another rounding.  Used only to measure the FP64 rounding floor."""

    name = "f64altfft"

    def spectral(self, kind: str, f):
        N = f.shape[0]
        key = ("full", kind, N)
        if key not in self._mult:
            k = np.arange(N)
            k = np.where(k <= N // 2, k, k - N)          # signed wavenumber of each bin
            m = multiplier(kind, N, np.abs(k).astype(float))
            self._mult[key] = np.where(k >= 0, m, np.conj(m))
        m = self._mult[key]
        fh = np.fft.fft(f, axis=0)
        fh = fh * (m[:, None] if f.ndim == 2 else m)
        return np.fft.ifft(fh, axis=0).real


class ArithAltSum(Arith):
    """The same FP64 arithmetic with the summation order of the products and of the
    dense solve reversed: matrix products sum over the inner index from the last term
    to the first, and A x = b is solved as (J A J)(J x) = J b with J the reversal, so
    that elimination runs from the last unknown to the first.  Used only to measure
    the FP64 rounding floor."""

    name = "f64altsum"

    def matmul(self, A, B):
        return A[:, ::-1] @ B[::-1]

    def lu_factor(self, A):
        return scipy.linalg.lu_factor(np.ascontiguousarray(A[::-1, ::-1]))

    def lu_solve(self, lu, B):
        return scipy.linalg.lu_solve(lu, np.ascontiguousarray(B[::-1]))[::-1]


class ArithAltInv(Arith):
    """The same FP64 arithmetic with every dense solve A x = b done through the explicit
    inverse, x = inv(A) b (inv from the same pivoted LU): mathematically the same
    solution, rounded differently (the inverse's own rounding, then one product).  Used
    only to measure the FP64 rounding floor."""

    name = "f64altinv"

    def lu_factor(self, A):
        return scipy.linalg.inv(A)

    def lu_solve(self, lu, B):
        return lu @ B


F64 = Arith()
F64ALT = ArithAlt()
F64ALT_FFT = ArithAltFFT()
F64ALT_SUM = ArithAltSum()
F64ALT_INV = ArithAltInv()


# --------------------------------------------------------------------------------
# spectral operators, Sec. 2.2 / App. A
# --------------------------------------------------------------------------------

def deriv(f, ar=F64):
    return ar.spectral("d", f)


def hilbert(f, ar=F64):
    return ar.spectral("h", f)


def proj(f, ar=F64):
    return ar.spectral("p", f)


def filt(f, ar=F64):
    return ar.spectral("f", f)


# --------------------------------------------------------------------------------
# cot branch formula, Sec. 2.2
# --------------------------------------------------------------------------------

def cot_half(x, y, ar=F64):
    """Real and imaginary parts of cot((x + i y)/2), by the two-branch formula of
    Sec. 2.2:  (cos x + cosh y)/(sin x + i sinh y) when cos x >= 0, otherwise
    (sin x - i sinh y)/(cosh y - cos x)."""
    cx, sx = ar.cos(x), ar.sin(x)
    chy, shy = ar.cosh_sinh(y)
    # branch 1: (cx + chy) (sx - i shy) / (sx^2 + shy^2)
    num = cx + chy
    d1 = sx * sx + shy * shy
    # branch 2: (sx - i shy) / (chy - cx)
    d2 = chy - cx
    pos = ar.ge0(cx)
    # guard the unused branch against 0/0 (it is discarded by `where`)
    one = ar.const(1.0)
    d1s = ar.where(pos, d1, one)
    d2s = ar.where(pos, one, d2)
    re = ar.where(pos, num * sx / d1s, sx / d2s)
    im = ar.where(pos, -num * shy / d1s, -shy / d2s)
    return re, im


# --------------------------------------------------------------------------------
# DtN operator, Sec. 2.1-2.2, App. A
# --------------------------------------------------------------------------------

def surface_height(eta, h):
    """Absolute surface height: h + eta at finite depth (bottom at y = 0), else eta."""
    return eta if math.isinf(h) else eta + h


def assemble(eta, h, ar=F64):
    """Collocation matrices of eq. (fred) and (G) on the uniform grid.

    Returns A = I/2 + K/N and Gm = G/N with K = K1 + K2, G = G1 + G2 as in (K1K2),
    reading R1 (minus sign on the image terms) and R2.  Row index i <-> alpha,
    column index j <-> beta.
    """
    N = eta.shape[0]
    alpha = ar.grid(N)
    et = surface_height(eta, h)
    ex = deriv(eta, ar)            # eta'  (Im zeta')
    exx = deriv(ex, ar)            # eta'' (Im zeta'')
    # zeta = alpha + i et, zeta' = 1 + i ex, zeta'' = i exx
    x = alpha[:, None] - alpha[None, :]
    y = et[:, None] - et[None, :]
    # off-diagonal terms only: park the diagonal at x = pi (finite values, overwritten
    # below by the regularised limits)
    xo = x.copy()
    for i in range(N):
        xo[i, i] = ar.pi
    cre, cim = cot_half(xo, y, ar)
    # cot((alpha_i - alpha_j)/2) / 2: real; used only in G1 (R2)
    c0re, _ = cot_half(xo, 0 * x, ar)
    c0 = c0re / 2
    # K1_ij = Im{ zeta'_j / 2 * C_ij } = (1/2)(cim + ex_j cre)
    K = (cim + ex[None, :] * cre) / 2
    # G1_ij = Re{ zeta'_i / 2 * C_ij } - cot((alpha_i-alpha_j)/2)/2 = (1/2)(cre - ex_i cim) - c0
    G = (cre - ex[:, None] * cim) / 2 - c0
    # diagonal limits: K1_ii = -Im{zeta''/(2 zeta')}, G1_ii = Re{zeta''/(2 zeta')}
    # zeta''/zeta' = i exx (1 - i ex)/(1 + ex^2) = (exx ex + i exx)/(1 + ex^2)
    den = 1 + ex * ex
    kd = -(exx / den) / 2
    gd = (exx * ex / den) / 2
    for i in range(N):
        K[i, i] = kd[i]
        G[i, i] = gd[i]
    if not math.isinf(h):
        # image terms with conj(zeta_j): x = alpha_i - alpha_j, y = et_i + et_j (all i, j)
        yb = et[:, None] + et[None, :]
        dre, dim = cot_half(x, yb, ar)
        # K2_ij = -Im{ conj(zeta'_j)/2 * D_ij } = -(1/2)(dim - ex_j dre)
        K = K - (dim - ex[None, :] * dre) / 2
        # G2_ij = -Re{ zeta'_i / 2 * D_ij } = -(1/2)(dre - ex_i dim)
        G = G - (dre - ex[:, None] * dim) / 2
    A = K / N
    for i in range(N):
        A[i, i] = A[i, i] + ar.const(0.5)
    Gm = G / N
    return A, Gm


class DtN:
    """Dirichlet-Neumann operator for one surface: assemble, factor once, apply to
    any number of right-hand sides (Sec. 3.3: one LU per stage, one back-solve per
    column)."""

    def __init__(self, eta, h, ar=F64):
        self.ar = ar
        self.A, self.Gm = assemble(eta, h, ar)
        self.lu = ar.lu_factor(self.A)

    def solve_mu(self, psi):
        return self.ar.lu_solve(self.lu, psi)

    def apply(self, psi):
        """G psi = (1/2) H gamma + Gm gamma, gamma = d mu / d alpha, A mu = psi  (eq. (G))."""
        ar = self.ar
        mu = self.solve_mu(psi)
        gam = deriv(mu, ar)
        return hilbert(gam, ar) / 2 + ar.matmul(self.Gm, gam), mu


def dtn_flat_symbol(k, h):
    """G e^{ikx} = |k| tanh(|k| h) e^{ikx} on the flat surface (Sec. 4.1)."""
    k = abs(k)
    return k if math.isinf(h) else k * math.tanh(k * h)


# --------------------------------------------------------------------------------
# right-hand sides: eq. (ww) for the base, App. B for the variational columns
# --------------------------------------------------------------------------------

def rhs(eta, phi, Qe, Qp, h, tau, g, ar=F64, want_aux=False):
    """F(q) and DF(q) Qdot for the augmented system (q:qdot), all filtered (R7).

    eta, phi: (N,) base; Qe, Qp: (N, M) variational columns or None.
    Returns (eta_t, phi_t, Qe_t, Qp_t).
    """
    N = eta.shape[0]
    dtn = DtN(eta, h, ar)
    ex = deriv(eta, ar)
    ps = deriv(phi, ar)                      # varphi'
    M = 0 if Qe is None else Qe.shape[1]
    # base Dirichlet data is phi itself; columns: psi_dot = phi_dot - phi_y eta_dot (l4)
    # so the base solve comes first (v is needed for the columns)
    Gphi, _ = dtn.apply(phi)
    den = 1 + ex * ex
    u = (ps - ex * Gphi) / den               # phi_x  (uv:from:G)
    v = (ex * ps + Gphi) / den               # phi_y
    eta_t = Gphi                             # phi_y - eta_x phi_x = G phi
    curv = deriv(ex / ar.sqrt(den), ar)
    phi_t = proj(v * eta_t - u * u / 2 - v * v / 2 - g * eta + tau * curv, ar)
    eta_t = filt(eta_t, ar)
    phi_t = filt(phi_t, ar)
    if M == 0:
        out = (eta_t, phi_t, None, None)
    else:
        psid = Qp - v[:, None] * Qe                              # (l4)
        Gpsid, _ = dtn.apply(psid)                               # G psi_dot
        Qe_t = Gpsid - deriv(Qe * u[:, None], ar)                # (l5a)
        dpsid = deriv(psid, ar)
        w3 = (den * ar.sqrt(den))                                # (1 + eta_x^2)^{3/2}
        tens = deriv(deriv(Qe, ar) / w3[:, None], ar)
        Qp_t = proj(-deriv(Qe * (u * v)[:, None], ar) - u[:, None] * dpsid
                    + v[:, None] * Gpsid - g * Qe + tau * tens, ar)   # (l6), (l6a)
        out = (eta_t, phi_t, filt(Qe_t, ar), filt(Qp_t, ar))
    if want_aux:
        return out, dict(u=u, v=v, Gphi=Gphi, dtn=dtn)
    return out


# --------------------------------------------------------------------------------
# DOP853 march to T/4, Sec. 2.2
# --------------------------------------------------------------------------------

def dop853_tableau():
    """Dormand-Prince 8(5,3) coefficients (Hairer, Norsett & Wanner, Solving ODEs I),
    12 stages for the 8th-order update, taken from SciPy's published table."""
    from scipy.integrate._ivp import dop853_coefficients as d
    s = d.N_STAGES
    return np.array(d.A[:s, :s], dtype=float), np.array(d.B, dtype=float), \
        np.array(d.C[:s], dtype=float)


def march(eta0, phi0, Qe0, Qp0, h, tau, g, T, nsteps, ar=F64, tableau=None, callback=None):
    """Evolve (q, Qdot) with nsteps fixed DOP853 steps of dt = T/(4 nsteps).

    Columns use the base stage values of the same stage (eq. (q:qdot)).  The filter is
    applied to every right-hand side and to the solution after every step.
    """
    a, b, c = tableau if tableau is not None else dop853_tableau()
    s = len(b)
    dt = ar.const(T) / (4 * nsteps)
    y = [eta0, phi0, Qe0, Qp0]
    has_cols = Qe0 is not None
    for n in range(nsteps):
        ks = []
        for i in range(s):
            Y = list(y)
            for j in range(i):
                if a[i, j] != 0.0:
                    aij = ar.const(a[i, j]) * dt
                    Y = [Y[q] + aij * ks[j][q] if ks[j][q] is not None else None
                         for q in range(4)]
            ks.append(rhs(Y[0], Y[1], Y[2], Y[3], h, tau, g, ar))
        ynew = list(y)
        for i in range(s):
            if b[i] != 0.0:
                bi = ar.const(b[i]) * dt
                ynew = [ynew[q] + bi * ks[i][q] if ks[i][q] is not None else None
                        for q in range(4)]
        y = [filt(ynew[0], ar), filt(ynew[1], ar),
             filt(ynew[2], ar) if has_cols else None,
             filt(ynew[3], ar) if has_cols else None]
        if callback is not None:
            callback(n + 1, y)
    return y


def shoot_eval(N, h, tau, g, basis, q_fixed, params, T, nsteps, jacobian=True,
               ar=F64, tableau=None):
    """r, J, drdT, f of the T/4 shooting problem (eq. (f:phi), (Jik), (dfdT)).

    basis: (2N, M); q0 = q_fixed + basis @ params; Qdot(0) = basis.
    Returns dict(r, J (N, M) or None, drdT, f, eta, phi).
    """
    basis = ar.asarray(basis)
    q0 = ar.asarray(q_fixed) + ar.matmul(basis, ar.asarray(params))
    eta0, phi0 = q0[:N], q0[N:]
    if jacobian:
        Qe0, Qp0 = basis[:N, :], basis[N:, :]
    else:
        Qe0 = Qp0 = None
    eta, phi, Qe, Qp = march(eta0, phi0, Qe0, Qp0, h, tau, g, T, nsteps, ar, tableau)
    w = 1 / ar.sqrt(ar.const(N))
    r = w * phi
    (_, phi_t, _, _) = rhs(eta, phi, None, None, h, tau, g, ar)
    drdT = w * phi_t / 4
    f = ar.sum(r * r) / 2
    return dict(r=r, J=(w * Qp) if jacobian else None, drdT=drdT, f=f, eta=eta, phi=phi)


def shoot_gradient(res):
    """grad_c f = J^T r and df/dT = drdT . r (reading R9)."""
    J, r = res["J"], res["r"]
    return J.T @ r, math.fsum(res["drdT"] * r)


def energy(eta, phi, h, tau, g, ar=F64):
    """E = (2 pi / N) sum[ phi G phi / 2 + g eta^2 / 2 + tau (sqrt(1 + eta_x^2) - 1) ]
    (Sec. 4.4 energy monitor, with the surface-tension energy added, reading R12)."""
    N = eta.shape[0]
    Gphi, _ = DtN(eta, h, ar).apply(phi)
    ex = deriv(eta, ar)
    e = phi * Gphi / 2 + g * eta * eta / 2 + tau * (ar.sqrt(1 + ex * ex) - 1)
    return 2 * ar.pi / N * ar.sum(e)


def stability_poly_coeffs(tableau=None):
    """beta_j with R(z) = sum_j beta_j z^j for the explicit tableau:
    beta_0 = 1, beta_j = b^T A^{j-1} 1 (used by the linear-propagator pin)."""
    a, b, c = tableau if tableau is not None else dop853_tableau()
    s = len(b)
    beta = [1.0]
    v = np.ones(s)
    for j in range(1, s + 1):
        beta.append(float(b @ v))
        v = a @ v
    return np.array(beta)
