"""Seeded synthetic workloads shaped like the standing-wave runs of Wilkening & Yu,
"Overdetermined shooting methods for computing standing water waves with spectral
accuracy" (Sec. 2.3 symmetric standing waves, Sec. 3.1 cosine-mode parametrisation,
Sec. 4.7 problem sizes).

This module only draws inputs: grid size, depth, surface tension, gravity, period,
step count, the parameter vector c and the basis that maps c to the initial state
q0 = q_fixed + basis @ c.  It holds none of the method's arithmetic, and is the one
module shared by the CPU reference and the GPU path.

Conventions (the paper leaves these open; the readings are listed with the design
notes):
  * the grid is alpha_j = 2 pi j / N, j = 0..N-1 (uniform mesh, xi(alpha) = alpha);
  * `surface` / eta is the displacement from the still level; at finite depth h the
    absolute surface height is h + eta (bottom at y = 0);
  * parameter k (k = 1..M) multiplies cos(k alpha) in the initial surface eta_0,
    and phi_0 = 0;
  * T is the full period and the march goes to T/4; T is the linear period of the
    k = 1 mode, 2 pi / sqrt((g + tau) tanh h)  (infinite depth: tanh -> 1);
  * random mode amplitudes a_k ~ Normal(0, std = 1e-3 * 2**-k) for k = 2..16 from
    numpy PCG64 seeded with 1210 + config index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

INF = math.inf


@dataclass
class Workload:
    name: str
    N: int
    h: float          # mean depth; math.inf for infinite depth
    tau: float        # surface tension / density
    g: float
    M: int            # number of parameters = Jacobian columns
    T: float          # full period; the march goes to T/4
    nsteps: int
    params: np.ndarray = field(repr=False)   # (M,)
    basis: np.ndarray = field(repr=False)    # (2N, M): rows 0..N-1 eta part, N..2N-1 phi part
    q_fixed: np.ndarray = field(repr=False)  # (2N,)
    ckpt_every: int = 16
    description: str = ""
    # time segments on non-uniform meshes (dicts with N, nsteps, theta, rho, refine_at;
    # the first N is the basis grid), or None for one uniform segment
    segments: list | None = field(default=None, repr=False)

    @property
    def R(self) -> int:
        return self.M + 1


def grid(N: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(N) / N


def linear_period(h: float, tau: float, g: float = 1.0, k: int = 1) -> float:
    """Linear standing-wave period of mode k (input choice for T)."""
    th = 1.0 if math.isinf(h) else math.tanh(k * h)
    return 2.0 * math.pi / math.sqrt((g + tau * k * k) * k * th)


def cosine_basis(N: int, M: int) -> np.ndarray:
    """Column k-1 = (cos(k alpha), 0): parameter k moves the eta-mode k of q0."""
    a = grid(N)
    B = np.zeros((2 * N, M))
    for k in range(1, M + 1):
        B[:N, k - 1] = np.cos(k * a)
    return B


def paper_basis(N: int, M: int) -> np.ndarray:
    """Standing-wave parametrisation of Sec. 3.1: c_k sets the k-th Fourier mode of
    eta (even k) or phi (odd k) with hat q_{+-k} = c_k, i.e. basis 2 cos(k alpha)."""
    a = grid(N)
    B = np.zeros((2 * N, M))
    for k in range(1, M + 1):
        if k % 2 == 0:
            B[:N, k - 1] = 2.0 * np.cos(k * a)
        else:
            B[N:, k - 1] = 2.0 * np.cos(k * a)
    return B


def _modes(rng: np.random.Generator, a1: float, M: int, kmax: int = 16) -> np.ndarray:
    p = np.zeros(M)
    p[0] = a1
    for k in range(2, min(kmax, M) + 1):
        p[k - 1] = rng.normal(0.0, 1e-3 * 2.0 ** (-k))
    return p


def c1() -> Workload:
    N, M = 64, 8
    p = np.zeros(M)
    p[0] = 0.01
    return Workload("c1_fp64_inf_N64", N, INF, 0.0, 1.0, M, 2.0 * math.pi, 64, p,
                    cosine_basis(N, M), np.zeros(2 * N),
                    description="infinite depth, N=64, eta0=0.01cos x, phi0=0, 64 RK8 steps "
                                "to T/4 with T=2pi, M=8 cosine-mode parameters")


def c2() -> Workload:
    rng = np.random.default_rng(1210 + 2)
    N, M, h, tau = 256, 64, 1.0, 0.0
    return Workload("c2_fp64_h1_N256", N, h, tau, 1.0, M, linear_period(h, tau), 300,
                    _modes(rng, 0.05, M), cosine_basis(N, M), np.zeros(2 * N),
                    description="h=1, tau=0, N=256, a1=0.05 + seeded modes 2..16, M=64, 300 steps")


def c3() -> Workload:
    rng = np.random.default_rng(1210 + 3)
    N, M, h, tau = 1024, 128, 0.5, 0.02
    return Workload("c3_h0.5_tau0.02_N1024_M128", N, h, tau, 1.0, M, linear_period(h, tau), 600,
                    _modes(rng, 0.05, M), cosine_basis(N, M), np.zeros(2 * N),
                    description="h=0.5, tau=0.02, N=1024, M=128, 600 steps (precision form)")


def c4() -> Workload:
    rng = np.random.default_rng(1210 + 4)
    N, M = 512, 256
    return Workload("c4_inf_N512_M256", N, INF, 0.0, 1.0, M, 2.0 * math.pi, 800,
                    _modes(rng, 0.2, M), cosine_basis(N, M), np.zeros(2 * N),
                    ckpt_every=16,
                    description="infinite depth, N=512, 256 cosine-mode parameters, a1=0.2, "
                                "800 steps, adjoint with checkpoints every 16 steps")


def c6() -> Workload:
    """Two time segments on non-uniform meshes, sized like the double-precision mesh
    parameters of Table tab:param:OA (solution A there: theta = (0.2, 0.8), rho = (1.0,
    0.4), 768 then 1024 grid points, 24 then 144 steps, 200 parameters); the mesh of the
    second segment is finest near x = pi.  Infinite depth, a1 = 0.15 with the seeded modes
    2..16, T = 2 pi."""
    rng = np.random.default_rng(1210 + 6)
    N, M = 768, 200
    segs = [dict(N=768, nsteps=24, theta=0.2, rho=1.0, refine_at=0),
            dict(N=1024, nsteps=144, theta=0.8, rho=0.4, refine_at=0)]
    return Workload("c6_inf_N768-1024_M200_segments", N, INF, 0.0, 1.0, M, 2.0 * math.pi, 168,
                    _modes(rng, 0.15, M), cosine_basis(N, M), np.zeros(2 * N), segments=segs,
                    description="two segments (theta 0.2, 0.8; rho 1.0, 0.4; N 768, 1024; 24 + 144 "
                                "steps), infinite depth, a1=0.15, M=200")


C5_SIZES = (256, 384, 512, 768, 1024, 1536, 2048)


def c5(n_inst: int = 32, seed: int = 1210 + 5, nsteps_cap: int | None = None) -> list[Workload]:
    """Batch of continuation instances of uneven N, depth, tension, amplitude and M.

    nsteps is the linear-stability step count for the filtered RK8 march (largest
    resolved mode), times 1.1, supplied by the caller through `nsteps_for`; here a
    conservative CFL-like estimate is used: dt * omega_max <= 4.5 with omega_max the
    fastest filtered linear frequency on the grid.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        N = int(rng.choice(C5_SIZES))
        h = INF if rng.uniform() < 0.25 else float(rng.uniform(0.05, 3.0))
        tau = float(rng.uniform(0.0, 0.05))
        a1 = float(rng.uniform(0.01, 0.4))
        if not math.isinf(h):
            a1 = min(a1, 0.2 * h)
        M = int(rng.integers(32, 257))
        M = max(1, min(M, N // 2))
        T = linear_period(h, tau)
        th = lambda k: 1.0 if math.isinf(h) else math.tanh(k * h)
        wmax = max(math.sqrt((1.0 + tau * k * k) * k * th(k)) *
                   math.exp(-36.0 * (k / (N / 2)) ** 36) for k in range(1, N // 2 + 1))
        nsteps = int(math.ceil(1.1 * (T / 4.0) * wmax / 4.5))
        nsteps = max(nsteps, 16)
        if nsteps_cap is not None:
            nsteps = min(nsteps, nsteps_cap)
        out.append(Workload(f"c5_{i:02d}_N{N}", N, h, tau, 1.0, M, T, nsteps,
                            _modes(rng, a1, M), cosine_basis(N, M), np.zeros(2 * N),
                            description="batched continuation instance"))
    return out


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c6": c6}


def initial_state(w: Workload) -> tuple[np.ndarray, np.ndarray]:
    """q0 = q_fixed + basis @ params, split into (eta0, phi0)."""
    q0 = w.q_fixed + w.basis @ w.params
    return q0[:w.N].copy(), q0[w.N:].copy()


def random_surface(N: int, seed: int, amp: float = 0.05, kmax: int = 12) -> np.ndarray:
    """Smooth random even/odd surface (displacement) with decaying modes."""
    rng = np.random.default_rng(seed)
    a = grid(N)
    eta = np.zeros(N)
    for k in range(1, kmax + 1):
        eta += amp * 2.0 ** (1 - k) * (rng.normal() * np.cos(k * a) + rng.normal() * np.sin(k * a))
    return eta


def steep_surface(N: int, amp: float = 0.15, k: int = 20) -> np.ndarray:
    """Under-resolved steep surface amp cos(k a) + 0.02 sin(3 a): at N = 64 the slopes
    reach 3 and A loses column dominance, so that elimination with partial pivoting
    interchanges rows (the pivoting fallback's test input)."""
    a = grid(N)
    return amp * np.cos(k * a) + 0.02 * np.sin(3 * a)


def random_rhs(N: int, R: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((N, R)))
