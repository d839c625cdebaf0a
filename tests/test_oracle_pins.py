"""Pins of the CPU reference against what the paper and the mathematics fix.

Each test checks the reference (oracle/) against something other than itself:
closed forms, printed values, invariants, brute force or an independent route.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest

from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(N):
    return 2 * np.pi * np.arange(N) / N


# ---------------------------------------------------------------- cot formula (Sec. 2.2)

def test_cot_branch_formula_matches_complex_tangent():
    rng = np.random.default_rng(0)
    x = rng.uniform(-7, 7, 4000)
    y = rng.uniform(-3, 3, 4000)
    keep = np.abs(np.sin((x + 1j * y) / 2)) > 1e-3
    x, y = x[keep], y[keep]
    re, im = O.cot_half(x, y)
    ref = np.array([1 / cmath.tan(complex(a, b) / 2) for a, b in zip(x, y)])
    err = np.abs(re + 1j * im - ref) / np.abs(ref)
    assert err.max() < 4e-15


# ---------------------------------------------------------------- spectral operators

def test_spectral_symbols_against_naive_dft():
    N = 24
    rng = np.random.default_rng(1)
    f = rng.standard_normal(N)
    a = _grid(N)
    ks = np.arange(-N // 2 + 1, N // 2 + 1)
    fh = np.array([np.sum(f * np.exp(-1j * k * a)) for k in ks]) / N

    def synth(mult):
        return np.real(sum(m * c * np.exp(1j * k * a) for k, m, c in zip(ks, mult, fh)))

    nyq = ks == N // 2
    dref = synth(np.where(nyq, 0, 1j * ks))
    href = synth(np.where(nyq, 0, -1j * np.sign(ks)))
    pref = synth(np.where(ks == 0, 0, 1.0))
    fref = synth(np.exp(-36.0 * (np.abs(ks) / (N / 2)) ** 36))
    for got, ref in ((O.deriv(f), dref), (O.hilbert(f), href), (O.proj(f), pref), (O.filt(f), fref)):
        assert np.abs(got - ref).max() < 1e-13


# ---------------------------------------------------------------- DtN (Sec. 2.1, App. A)

@pytest.mark.parametrize("h,N", [(math.inf, 64), (1.0, 64), (0.3, 128)])
def test_flat_surface_dtn_symbol(h, N):
    """G e^{ikx} = k tanh(kh) e^{ikx} on the flat surface (Sec. 4.1, eq. (lin));
    (N - k) h large enough that trapezoid aliasing of the image kernel is < 1e-16."""
    a = _grid(N)
    d = O.DtN(np.zeros(N), h)
    if math.isinf(h):
        assert np.array_equal(d.A, 0.5 * np.eye(N))
    for k in (1, 2, 5, 11):
        psi = np.cos(k * a) + 0.5 * np.sin(k * a)
        G, _ = d.apply(psi)
        assert np.abs(G - O.dtn_flat_symbol(k, h) * psi).max() < 2e-13 * k


def _harmonic(eta, h, k, a, ex):
    """Closed-form DtN pair: phi = e^{ky} cos kx (infinite depth) or cosh(ky) cos kx
    (bottom at y = 0) is harmonic with phi_y = 0 at the bottom; its surface trace psi
    and G psi = phi_y - eta_x phi_x on y = surface height."""
    if math.isinf(h):
        s = eta
        psi = np.exp(k * s) * np.cos(k * a)
        phx = -k * np.exp(k * s) * np.sin(k * a)
        phy = k * np.exp(k * s) * np.cos(k * a)
    else:
        s = eta + h
        psi = np.cosh(k * s) * np.cos(k * a)
        phx = -k * np.cosh(k * s) * np.sin(k * a)
        phy = k * np.sinh(k * s) * np.cos(k * a)
    return psi, phy - ex * phx


@pytest.mark.parametrize("h", [math.inf, 1.0, 0.5])
@pytest.mark.parametrize("k", [1, 3])
def test_dtn_exact_on_nonflat_surface(h, k):
    """Full nonlinear kernel (K1, K2, G1, G2, diagonal limits, solve, gamma = mu',
    Hilbert term) against an exact harmonic function on a non-flat surface."""
    N = 128
    a = _grid(N)
    eta = 0.1 * np.cos(a) + 0.03 * np.sin(2 * a) + 0.01 * np.cos(3 * a)
    ex = -0.1 * np.sin(a) + 0.06 * np.cos(2 * a) - 0.03 * np.sin(3 * a)
    psi, Gex = _harmonic(eta, h, k, a, ex)
    G, _ = O.DtN(eta, h).apply(psi)
    assert np.abs(G - Gex).max() / np.abs(Gex).max() < 1e-12


def test_dtn_exact_crest_surface_converges_spectrally():
    """Sharper surface: the error must fall spectrally with N (trapezoid rule on
    smooth periodic kernels)."""
    errs = []
    for N in (32, 64, 128):
        a = _grid(N)
        eta = 0.25 * np.cos(a) + 0.06 * np.cos(2 * a)
        ex = -0.25 * np.sin(a) - 0.12 * np.sin(2 * a)
        psi, Gex = _harmonic(eta, 0.8, 2, a, ex)
        G, _ = O.DtN(eta, 0.8).apply(psi)
        errs.append(np.abs(G - Gex).max() / np.abs(Gex).max())
    assert errs[0] > errs[1] > errs[2] or errs[2] < 1e-12
    assert errs[2] < 1e-11


def test_dtn_mass_and_constants():
    """G 1 = 0 and the mean of G psi vanishes (int G phi dx = 0)."""
    N = 64
    a = _grid(N)
    eta = W.random_surface(N, 3, amp=0.08)
    for h in (math.inf, 0.7):
        d = O.DtN(eta, h)
        G1, _ = d.apply(np.ones(N))
        assert np.abs(G1).max() < 1e-12
        Gp, _ = d.apply(np.sin(3 * a) + np.cos(a) ** 2)
        assert abs(Gp.mean()) < 1e-13


def test_craig_sulem_first_order_shape_derivative():
    """[G(h + eps e) - G(h - eps e)] psi / (2 eps) -> -d(e d psi) - G0(e G0 psi)."""
    N, h, eps = 64, 1.0, 1e-4
    a = _grid(N)
    e = np.cos(a) + 0.3 * np.sin(2 * a)
    psi = np.cos(2 * a) + 0.2 * np.sin(3 * a)
    Gp, _ = O.DtN(eps * e, h).apply(psi)
    Gm, _ = O.DtN(-eps * e, h).apply(psi)
    d0 = O.DtN(np.zeros(N), h)
    G0psi, _ = d0.apply(psi)
    G0eG0, _ = d0.apply(e * G0psi)
    ref = -O.deriv(e * O.deriv(psi)) - G0eG0
    got = (Gp - Gm) / (2 * eps)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-7


# ---------------------------------------------------------------- tableau (Sec. 2.2)

def test_dop853_order_conditions():
    a, b, c = O.dop853_tableau()
    assert np.allclose(np.triu(a), 0)                     # explicit
    assert np.allclose(a.sum(axis=1), c, atol=2e-15)
    for q in range(8):                                    # bushy trees
        assert abs(b @ c ** q - 1 / (q + 1)) < 1e-14
    for q in range(6):                                    # sum_i b_i c_i^q (A c)_i = 1/(2(q+3))
        assert abs(b @ (c ** q * (a @ c)) - 1 / (2 * (q + 3))) < 1e-14
    for q in range(5):                                    # sum_i b_i c_i^q (A c^2)_i = 1/(3(q+4))
        assert abs(b @ (c ** q * (a @ c ** 2)) - 1 / (3 * (q + 4))) < 1e-14
    beta = O.stability_poly_coeffs((a, b, c))             # R(z) = e^z + O(z^9)
    for j in range(9):
        assert abs(beta[j] - 1 / math.factorial(j)) < 1e-15
    assert abs(beta[9] - 1 / math.factorial(9)) > 1e-9    # order exactly 8


# ---------------------------------------------------------------- linear dynamics

def _propagator(k, h, tau, g, N, T, nsteps):
    """Discrete, filtered linear propagator of mode k at the flat rest state:
    per step  sigma_k R(dt sigma_k L_k),  R the stability polynomial of the tableau
    (evaluated from its coefficients, not by running stages)."""
    beta = O.stability_poly_coeffs()
    dt = T / (4 * nsteps)
    sig = math.exp(-36.0 * (k / (N / 2)) ** 36)
    lam = O.dtn_flat_symbol(k, h)
    L = np.array([[0.0, lam], [-(g + tau * k * k), 0.0]])
    Z = dt * sig * L
    R = np.zeros((2, 2))
    P = np.eye(2)
    for bj in beta:
        R += bj * P
        P = P @ Z
    S = sig * R
    return np.linalg.matrix_power(S, nsteps)


@pytest.mark.parametrize("h,tau", [(math.inf, 0.0), (1.5, 0.02)])
def test_rest_state_jacobian_is_discrete_linear_propagator(h, tau):
    """P7: at the flat rest state the Jacobian columns are the filtered discrete
    propagator of each mode, including the filter at high k."""
    N, nsteps = 32, 6
    T = W.linear_period(h, tau)
    M = 12
    basis = W.cosine_basis(N, M)
    res = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), np.zeros(M), T, nsteps)
    a = _grid(N)
    w = 1 / math.sqrt(N)
    assert np.abs(res["r"]).max() == 0.0
    for k in range(1, M + 1):
        S = _propagator(k, h, tau, 1.0, N, T, nsteps)
        ref = w * S[1, 0] * np.cos(k * a)
        assert np.abs(res["J"][:, k - 1] - ref).max() < 1e-14 * max(1.0, abs(S[1, 0]))


def test_golden_linear_periods_rest_at_quarter_period():
    """Printed linear periods (Sec. 4.1, 4.5, 4.6): from (eta, phi) = (0, cos x) the
    linear flow is at rest at T/4 (phi = 0), with eta = (A/B) cos x."""
    cases = json.load(open(os.path.join(GOLDEN, "linear_periods.json")))["cases"]
    for c in cases:
        h = math.inf if c["h"] == "inf" else float(c["h"])
        tau, T = float(c["tau"]), float(c["T"])
        N = 256 if (not math.isinf(h) and h < 0.2) else 32
        nsteps = 24
        basis = np.zeros((2 * N, 1))
        a = _grid(N)
        basis[N:, 0] = np.cos(a)
        q = np.zeros(2 * N)
        eta, phi, Qe, Qp = O.march(q[:N], q[N:], basis[:N], basis[N:], h, tau, 1.0, T, nsteps)
        tol = 10.0 ** (1 - c["digits"]) * 2
        # phi_dot(T/4) = cos(w T/4) cos x ~ 0 to the printed digits of T
        assert np.abs(Qp).max() < tol, c
        ratio = math.sqrt(O.dtn_flat_symbol(1, h) / (1.0 + tau))
        if "A_over_B" in c:
            assert abs(ratio - math.sqrt(math.tanh(1.0))) < 1e-15
        assert np.abs(Qe[:, 0] - ratio * np.cos(a)).max() < tol * 3, c


# ---------------------------------------------------------------- nonlinear invariants

@pytest.mark.parametrize("h,tau,amp,N,nsteps", [(math.inf, 0.0, 0.01, 64, 64),
                                                 (1.0, 0.02, 0.08, 64, 48)])
def test_energy_conservation(h, tau, amp, N, nsteps):
    """Energy is conserved to 12+ digits (Sec. 2.2, Sec. 4.4 report 14 typically)."""
    a = _grid(N)
    eta0 = amp * np.cos(a) + 0.2 * amp * np.cos(2 * a)
    phi0 = 0.3 * amp * np.cos(a)
    T = W.linear_period(h, tau)
    E0 = O.energy(eta0, phi0, h, tau, 1.0)
    eta, phi, _, _ = O.march(eta0, phi0, None, None, h, tau, 1.0, T, nsteps)
    E1 = O.energy(eta, phi, h, tau, 1.0)
    assert abs(E1 - E0) / abs(E0) < 1e-12
    assert np.abs(phi - phi0).max() > 1e-3 * amp    # the state really moved


def test_time_reversal_bitwise():
    """F(eta, -phi) = -S F(eta, phi) with S(eta, phi) = (eta, -phi): marching the
    reflected state forward equals reflecting the backward march, bit for bit."""
    N, nsteps, h, tau = 32, 4, 0.9, 0.01
    a = _grid(N)
    eta0 = 0.06 * np.cos(a) + 0.01 * np.sin(3 * a)
    phi0 = 0.02 * np.sin(a) + 0.01 * np.cos(2 * a)
    T = 7.0
    e1, p1, _, _ = O.march(eta0, -phi0, None, None, h, tau, 1.0, T, nsteps)
    e2, p2, _, _ = O.march(eta0, phi0, None, None, h, tau, 1.0, -T, nsteps)
    assert np.array_equal(e1, e2)
    assert np.array_equal(p1, -p2)
    # and the round trip recovers q0 to truncation error
    e3, p3, _, _ = O.march(e1, -p1, None, None, h, tau, 1.0, T, nsteps)
    assert np.abs(e3 - eta0).max() < 1e-7 and np.abs(p3 - phi0).max() < 1e-7


def test_even_data_stays_even():
    w = W.c1()
    res = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, 16)
    eta, phi = res["eta"], res["phi"]
    rev = lambda f: np.roll(f[::-1], 1)      # f(-x) on the grid
    for f in (eta, phi):
        assert np.abs(f - rev(f)).max() < 1e-15 + 1e-13 * np.abs(f).max()


# ---------------------------------------------------------------- Jacobian, T-derivative

def test_jacobian_matches_central_differences():
    """P11: variational columns (App. B) against central differences of r.  The
    variational equation is the discretised linearisation of the PDE, not the exact
    derivative of the discrete scheme; the two agree to the spatial discretisation
    error, which is below 1e-8 here (N = 48) and falls spectrally with N."""
    N, M, h, tau, nsteps = 48, 4, 1.0, 0.01, 8
    basis = W.cosine_basis(N, M)
    p = np.array([0.05, 0.01, -0.004, 0.002])
    T = W.linear_period(h, tau)
    res = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, T, nsteps)
    eps = 1e-5
    for k in range(M):
        d = np.zeros(M)
        d[k] = eps
        rp = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p + d, T, nsteps, jacobian=False)["r"]
        rm = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p - d, T, nsteps, jacobian=False)["r"]
        fd = (rp - rm) / (2 * eps)
        assert np.linalg.norm(fd - res["J"][:, k]) < 1e-7 * np.linalg.norm(res["J"][:, k])


def test_jacobian_phi_columns_match_central_differences():
    """Same with the paper's parametrisation (phi modes at odd k, eta at even k)."""
    N, M, h, tau, nsteps = 32, 3, math.inf, 0.0, 8
    basis = W.paper_basis(N, M)
    p = np.array([0.03, 0.004, -0.002])
    res = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, 2 * np.pi, nsteps)
    eps = 1e-5
    for k in range(M):
        d = np.zeros(M)
        d[k] = eps
        rp = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p + d, 2 * np.pi, nsteps, jacobian=False)["r"]
        rm = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p - d, 2 * np.pi, nsteps, jacobian=False)["r"]
        fd = (rp - rm) / (2 * eps)
        assert np.linalg.norm(fd - res["J"][:, k]) < 1e-7 * np.linalg.norm(res["J"][:, k])


def test_drdT_matches_difference_in_T():
    """drdT = phi_t(T/4) w / 4 against central differences in T; they agree to the
    time-truncation level (the discrete march depends on T through dt)."""
    N, M, h, tau, nsteps = 32, 1, 1.0, 0.0, 16
    basis = W.cosine_basis(N, M)
    p = np.array([0.05])
    T = W.linear_period(h, tau)
    res = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, T, nsteps, jacobian=False)
    eps = 1e-5
    rp = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, T + eps, nsteps, jacobian=False)["r"]
    rm = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, T - eps, nsteps, jacobian=False)["r"]
    fd = (rp - rm) / (2 * eps)
    assert np.linalg.norm(fd - res["drdT"]) < 1e-6 * np.linalg.norm(res["drdT"])


# ---------------------------------------------------------------- FP64 rounding floor

def test_fp64_reference_against_extended_precision():
    """P13: the FP64 reference agrees with the same scheme run in 34-digit arithmetic."""
    from oracle.xprec import MPArith, to_float
    mp = MPArith(34)
    N, M, h, tau, nsteps = 16, 2, 1.0, 0.01, 2
    basis = W.cosine_basis(N, M)
    p = np.array([0.05, 0.01])
    T = 7.0
    hi = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, T, nsteps, ar=mp)
    lo = O.shoot_eval(N, h, tau, 1.0, basis, np.zeros(2 * N), p, T, nsteps)
    er = np.linalg.norm(to_float(hi["r"]) - lo["r"]) / np.linalg.norm(lo["r"])
    eJ = np.linalg.norm(to_float(hi["J"]) - lo["J"]) / np.linalg.norm(lo["J"])
    assert er < 1e-13 and eJ < 1e-13
