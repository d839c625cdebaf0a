"""Pins of the mesh oracle (oracle/mesh_oracle.py): the non-uniform mesh x = xi(alpha)
of Sec. 2.2 eq. (xi), (rho:def) and the time segments with regridding, checked against
what the paper and the mathematics fix, not against the oracle itself:

  * eq. (rho:def): E(0), E(pi) and their ratio rho; xi(2 pi) = 2 pi; mean of E one;
    E = xi' and E' = E'' by central differences; xi^{-1}(xi(a)) = a;
  * rho = 1 reduces to the uniform-mesh oracle (the independent code of ww_oracle);
  * the flat-surface symbol |k| tanh(|k| h) on mapped grids (Sec. 4.1), where
    cos(k xi(alpha)) is not band-limited in alpha: spectral accuracy;
  * invariance under the parametrisation: the DtN of one curve on a mapped grid equals
    the uniform-grid DtN of the same curve, interpolated (catches any slip in zeta',
    zeta'', the 1/|xi'| factor or the alpha-regularisation of G1);
  * the regridding reproduces a band-limited function of x exactly from a uniform mesh;
  * a segmented march with a refined second segment: energy (R12) conserved, the
    x-mean of varphi (reading M1's projection) conserved, even data stays even, J
    against central differences (P11), two identical uniform segments equal one,
    and the objective weights (M3) against the x-integral on a fine grid;
  * small-amplitude standing wave on a mapped grid against the linear solution.
"""
import math

import numpy as np
import pytest

from oracle import mesh_oracle as MO
from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W


def test_mesh_closed_forms():
    for rho in (1.0, 0.6, 0.25, 0.09):
        for side in (MO.REFINE_PI, MO.REFINE_ZERO):
            m = MO.Mesh(48, rho, side)
            e0, epi = float(m.E_at(0.0)), float(m.E_at(np.pi))
            lo, hi = (epi, e0) if side == MO.REFINE_PI else (e0, epi)
            assert abs(lo - 8 * rho / (5 + 3 * rho)) < 1e-15
            assert abs(hi - 8 / (5 + 3 * rho)) < 1e-15
            assert abs(lo / hi - rho) < 1e-15
            assert abs(float(m.xi_at(2 * np.pi)) - 2 * np.pi) < 1e-14
            assert abs(m.E.mean() - 1.0) < 1e-15            # E is a degree-2 trig polynomial
            a = np.linspace(0.1, 6.0, 17)
            d = 1e-5
            assert np.max(np.abs((m.xi_at(a + d) - m.xi_at(a - d)) / (2 * d) - m.E_at(a))) < 1e-9
            assert np.max(np.abs((m.E_at(a + d) - m.E_at(a - d)) / (2 * d) - m.Ep_at(a))) < 1e-9
            assert np.all(np.diff(m.xi) > 0)
            assert np.max(np.abs(m.xi_inverse(m.xi) - m.alpha)) < 1e-14


def test_rho_one_is_the_uniform_oracle():
    N = 64
    rng = np.random.default_rng(3)
    a = 2 * np.pi * np.arange(N) / N
    eta = 0.05 * np.cos(a) + 1e-3 * rng.standard_normal(N)
    phi = 0.02 * np.sin(2 * a)
    Qe, Qp = rng.standard_normal((N, 3)), rng.standard_normal((N, 3))
    for h in (math.inf, 0.7):
        A0, G0 = O.assemble(eta, h)
        A1, G1 = MO.assemble_mapped(eta, h, MO.Mesh(N))
        assert np.max(np.abs(A0 - A1)) < 1e-15 and np.max(np.abs(G0 - G1)) < 1e-15
        for x, y in zip(O.rhs(eta, phi, Qe, Qp, h, 0.02, 1.0), MO.rhs_mapped(eta, phi, Qe, Qp, h, 0.02, 1.0, MO.Mesh(N))):
            assert np.max(np.abs(x - y)) < 1e-13


@pytest.mark.parametrize("h", [math.inf, 1.0])
@pytest.mark.parametrize("rho,side", [(0.5, MO.REFINE_PI), (0.2, MO.REFINE_PI), (0.3, MO.REFINE_ZERO)])
def test_flat_symbol_on_mapped_grids(h, rho, side):
    N = 256
    m = MO.Mesh(N, rho, side)
    d = MO.DtNMapped(np.zeros(N), h, m)
    for k in range(1, 7):
        for f in (np.cos, np.sin):
            phi = f(k * m.xi)
            G, _ = d.apply(phi)
            assert np.max(np.abs(G - O.dtn_flat_symbol(k, h) * phi)) < 2e-12, (k, f)


@pytest.mark.parametrize("h", [math.inf, 0.8])
def test_dtn_is_invariant_under_the_parametrisation(h):
    N = 256
    f_eta = lambda x: 0.05 * np.cos(x) + 0.01 * np.cos(2 * x) + 0.004 * np.cos(3 * x) + 0.002 * np.sin(x)
    f_phi = lambda x: 0.02 * np.cos(x) - 0.01 * np.sin(2 * x) + 0.003 * np.cos(4 * x)
    u = MO.Mesh(N)
    Gu, _ = O.DtN(f_eta(u.xi), h).apply(f_phi(u.xi))
    for rho, side in ((0.5, MO.REFINE_PI), (0.2, MO.REFINE_PI), (0.35, MO.REFINE_ZERO)):
        m = MO.Mesh(N, rho, side)
        Gm, _ = MO.DtNMapped(f_eta(m.xi), h, m).apply(f_phi(m.xi))
        assert np.max(np.abs(Gm - MO.trig_interp(Gu, m.xi))) < 1e-12, rho


def test_regrid_is_exact_from_a_uniform_mesh():
    f = lambda x: np.cos(3 * x) + 0.3 * np.sin(5 * x) + 0.1 - 0.2 * np.cos(16 * x)
    u = MO.Mesh(64)
    for new in (MO.Mesh(96, 0.4), MO.Mesh(72, 0.7, MO.REFINE_ZERO), MO.Mesh(64)):
        assert np.max(np.abs(MO.regrid(f(u.xi), u, new) - f(new.xi))) < 1e-13
    cols = np.stack([f(u.xi), 2 * f(u.xi)], axis=1)
    out = MO.regrid(cols, u, MO.Mesh(96, 0.4))
    assert np.max(np.abs(out[:, 1] - 2 * out[:, 0])) < 1e-14


def test_segment_rules():
    with pytest.raises(ValueError):
        MO.check_segments([dict(N=64, nsteps=1, theta=0.5, rho=1.0), dict(N=64, nsteps=1, theta=0.4, rho=1.0)])
    with pytest.raises(ValueError):   # refining at the expense of the other region
        MO.check_segments([dict(N=64, nsteps=1, theta=0.5, rho=1.0), dict(N=64, nsteps=1, theta=0.5, rho=0.5)])
    MO.check_segments([dict(N=64, nsteps=1, theta=0.5, rho=1.0), dict(N=80, nsteps=1, theta=0.5, rho=0.5)])


SEGS = [dict(N=64, nsteps=20, theta=0.3, rho=1.0, refine_at=0),
        dict(N=96, nsteps=40, theta=0.7, rho=0.5, refine_at=0)]


def _problem(N=64, M=4):
    a = 2 * np.pi * np.arange(N) / N
    basis = np.zeros((2 * N, M))
    for k in range(1, M + 1):
        basis[:N, k - 1] = np.cos(k * a)
    return basis, np.zeros(2 * N), np.array([0.05, 0.004, -0.002, 0.001])[:M]


@pytest.fixture(scope="module")
def segmented():
    basis, qf, params = _problem()
    return basis, qf, params, MO.shoot_eval_segments(64, math.inf, 0.0, 1.0, basis, qf, params, 2 * np.pi, SEGS)


def test_segmented_march_invariants(segmented):
    basis, qf, params, res = segmented
    q0 = qf + basis @ params
    e0 = MO.energy_mapped(q0[:64], q0[64:], math.inf, 0.0, 1.0, MO.Mesh(64))
    e1 = MO.energy_mapped(res["eta"], res["phi"], math.inf, 0.0, 1.0, res["mesh"])
    assert abs(e1 - e0) / e0 < 1e-12                          # R12 energy, through the regrid
    m = res["mesh"]
    assert abs(np.dot(m.E, res["phi"]) / m.N) < 1e-14         # x-mean of varphi (reading M1)
    phi, J = res["phi"], res["J"]
    assert np.max(np.abs(phi[1:] - phi[1:][::-1])) < 1e-14   # even data stays even (xi is odd)
    assert np.max(np.abs(J[1:] - J[1:][::-1])) < 1e-14
    # objective weights (M3): f = (1/(4 pi)) int varphi^2 dx, the integral on a fine
    # uniform grid of the interpolated state
    fine = MO.regrid(phi, m, MO.Mesh(4 * m.N))
    assert abs(res["f"] - 0.5 * np.mean(fine ** 2)) < 1e-12 * res["f"] + 1e-18


def test_segmented_jacobian_by_central_differences(segmented):
    basis, qf, params, res = segmented
    eps = 1e-5
    for k in range(len(params)):
        rs = []
        for sgn in (1, -1):
            p = params.copy()
            p[k] += sgn * eps
            rs.append(MO.shoot_eval_segments(64, math.inf, 0.0, 1.0, basis, qf, p, 2 * np.pi, SEGS, jacobian=False)["r"])
        fd = (rs[0] - rs[1]) / (2 * eps)
        assert np.linalg.norm(fd - res["J"][:, k]) / np.linalg.norm(res["J"][:, k]) < 1e-6, k


def test_identical_segments_equal_one_march():
    basis, qf, params = _problem()
    one = MO.shoot_eval_segments(64, 0.9, 0.01, 1.0, basis, qf, params, 7.0,
                                 [dict(N=64, nsteps=30, theta=1.0, rho=1.0)])
    two = MO.shoot_eval_segments(64, 0.9, 0.01, 1.0, basis, qf, params, 7.0,
                                 [dict(N=64, nsteps=10, theta=1 / 3, rho=1.0), dict(N=64, nsteps=20, theta=2 / 3, rho=1.0)])
    uni = O.shoot_eval(64, 0.9, 0.01, 1.0, basis, qf, params, 7.0, 30)
    for k in ("r", "J", "drdT"):
        assert np.max(np.abs(one[k] - two[k])) < 1e-14
        assert np.max(np.abs(one[k] - uni[k])) < 1e-14


@pytest.mark.parametrize("h", [math.inf, 1.0])
def test_linear_standing_wave_on_a_mapped_grid(h):
    """eta0 = a cos(k x), varphi0 = 0 at amplitude a = 1e-7: at T/4 of the linear period
    varphi = -(g a / omega) sin(omega T / 4) cos(k x), up to O(a) nonlinearity and the
    RK truncation error."""
    k, g, a = 2, 1.0, 1e-7
    om = math.sqrt(g * O.dtn_flat_symbol(k, h))
    T = 2 * math.pi / om
    segs = [dict(N=48, nsteps=16, theta=0.5, rho=1.0), dict(N=64, nsteps=16, theta=0.5, rho=0.6, refine_at=1)]
    x0 = MO.Mesh(48).xi
    qf = np.concatenate([a * np.cos(k * x0), np.zeros(48)])
    res = MO.shoot_eval_segments(48, h, 0.0, 1.0, np.zeros((96, 0)), qf, np.zeros(0), T, segs, jacobian=False)
    m = res["mesh"]
    exact = -(g * a / om) * math.sin(om * T / 4) * np.cos(k * m.xi)
    assert np.max(np.abs(res["phi"] - exact)) < 10 * a * np.max(np.abs(exact))   # relative 10 a (P6)


def test_sdc_on_one_uniform_segment_is_the_uniform_sdc_march():
    """rho = 1 (E = 1): the mapped SDC15 march of one segment equals the uniform SDC15
    oracle (a different right-hand-side code) to rounding."""
    from oracle import sdc_oracle as S
    N, M = 32, 2
    basis = W.cosine_basis(N, M)
    p = np.array([0.03, 0.002])
    q = np.zeros(2 * N)
    a = MO.shoot_eval_segments(N, math.inf, 0.0, 1.0, basis, q, p, 2 * math.pi,
                               [dict(N=N, nsteps=2, theta=1.0, rho=1.0)], scheme="sdc")
    b = S.shoot_eval_sdc(N, math.inf, 0.0, 1.0, basis, q, p, 2 * math.pi, 2)
    for k in ("r", "J", "drdT"):
        assert np.abs(a[k] - b[k]).max() < 1e-13 * np.abs(b[k]).max(), k


def test_sdc_segments_agree_with_dop853_segments():
    """Two segments (the second refined, rho = 0.6) marched by SDC15 and by DOP853 at steps
    that resolve the solution: the two time integrators agree."""
    N, M = 32, 2
    basis = W.cosine_basis(N, M)
    p = np.array([0.03, 0.002])
    q = np.zeros(2 * N)
    segs_s = [dict(N=32, nsteps=2, theta=0.3, rho=1.0), dict(N=48, nsteps=4, theta=0.7, rho=0.6)]
    segs_r = [dict(N=32, nsteps=16, theta=0.3, rho=1.0), dict(N=48, nsteps=40, theta=0.7, rho=0.6)]
    a = MO.shoot_eval_segments(N, math.inf, 0.0, 1.0, basis, q, p, 2 * math.pi, segs_s, scheme="sdc")
    b = MO.shoot_eval_segments(N, math.inf, 0.0, 1.0, basis, q, p, 2 * math.pi, segs_r)
    for k in ("r", "J"):
        e = np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()
        print(k, e)
        assert e < 1e-10, k
