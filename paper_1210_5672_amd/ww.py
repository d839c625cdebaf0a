"""Python binding of the gfx950 library (include/ww.h): argument marshalling only.

Every step of the path runs in the HIP kernels of libwwdtn.so; torch supplies device
memory and the stream.  The library must be built (paper_1210_5672_amd/build.py);
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwwdtn.so")

WW_FP64 = 0
WW_MIXED = 1
WW_STRICT = 2
WW_GMRES = 4
WW_FB_PIVOTED = 1
WW_FB_FP64 = 2
WW_FB_DIRECT = 4

_ERRORS = {
    -1: "WW_EINVAL", -2: "WW_ENOSETUP", -3: "WW_EHIP", -4: "WW_EDOMAIN",
    -5: "WW_ENONFINITE", -6: "WW_EPIVOT", -7: "WW_EREFINE", -8: "WW_ENOCONV",
}
LM_REASONS = {1: "f=0", 2: "c unchanged", 3: "roundoff: rejected", 4: "roundoff: max_stepsJ",
              5: "max_evals"}


class LmOpts(ctypes.Structure):
    _fields_ = [("f_tol", ctypes.c_double), ("g_tol", ctypes.c_double), ("df_tol", ctypes.c_double),
                ("delta0", ctypes.c_double), ("max_steps_J", ctypes.c_int), ("max_evals", ctypes.c_int)]


class BfgsOpts(ctypes.Structure):
    _fields_ = [("f_tol", ctypes.c_double), ("g_tol", ctypes.c_double), ("delta0", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("ckpt_every", ctypes.c_int)]


class BfgsReport(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("gnorm", ctypes.c_double), ("iters", ctypes.c_int),
                ("evals", ctypes.c_int), ("reason", ctypes.c_int), ("n_hist", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int)]


BFGS_REASONS = {1: "f_tol", 2: "g_tol", 3: "c unchanged", 4: "line search", 5: "max_iter"}


class Tuning(ctypes.Structure):
    """Launch and scheduling choices of a context (ww_tuning)."""
    _fields_ = [(n, ctypes.c_int) for n in ("lag", "lu_group", "lu_streams", "graph_parts", "minv_wgs",
                                             "blu_strip", "dtn_rows", "gemm_split", "asm_cw", "gemm_rows", "lag_fp32",
                                             "lag_sweeps")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Segment(ctypes.Structure):
    """One time segment on a non-uniform mesh (ww_segment)."""
    _fields_ = [("N", ctypes.c_int), ("nsteps", ctypes.c_int), ("theta", ctypes.c_double),
                ("rho", ctypes.c_double), ("refine_at", ctypes.c_int)]


REFINE_PI, REFINE_ZERO = 0, 1


class LmReport(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("delta", ctypes.c_double), ("evals_r", ctypes.c_int),
                ("evals_J", ctypes.c_int), ("reason", ctypes.c_int), ("n_hist", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int)]

EXPORTS = ["ww_create", "ww_destroy", "ww_set_stream", "ww_set_tableau", "dtn_setup",
           "dtn_solve_multi", "shoot_setup", "shoot_eval", "shoot_adjoint", "ww_last_error",
           "ww_version", "ww_profile", "ww_profile_read", "shoot_eval_batch", "ww_fallbacks",
           "ww_thin_svd", "ww_levmar", "ww_lm_default_opts", "ww_bfgs", "ww_bfgs_default_opts",
           "dtn_solve_multi_noalloc", "ww_next_fallback", "ww_get_tuning", "ww_set_tuning",
           "shoot_eval_segments", "dtn_setup_dd", "dtn_solve_multi_dd", "shoot_eval_sdc",
           "shoot_eval_sdc_dd", "shoot_eval_segments_sdc"]


class WWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = _ERRORS.get(code, str(code))


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libwwdtn.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1210_5672_amd/build.py")
    lib = ctypes.CDLL(path)
    P, I, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    DP = ctypes.POINTER(ctypes.c_double)
    lib.ww_create.argtypes = [ctypes.POINTER(P), I, I, U, P]
    lib.ww_destroy.argtypes = [P]
    lib.ww_destroy.restype = None
    lib.ww_set_stream.argtypes = [P, P]
    lib.ww_set_tableau.argtypes = [P, I, DP, DP, DP]
    lib.dtn_setup.argtypes = [P, P, D, D, I]
    lib.dtn_solve_multi.argtypes = [P, P, I, P, P]
    lib.dtn_solve_multi_noalloc.argtypes = [P, P, I, P, P]
    lib.ww_next_fallback.argtypes = [U, U, I]
    lib.ww_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.ww_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.ww_next_fallback.restype = U
    lib.shoot_setup.argtypes = [P, I, D, D, D, P, P, I]
    lib.shoot_eval.argtypes = [P, P, D, I, P, P, P, DP]
    lib.shoot_adjoint.argtypes = [P, P, D, I, I, P, DP, DP]
    lib.shoot_eval_segments.argtypes = [P, P, D, I, ctypes.POINTER(Segment), P, P, P, DP]
    lib.shoot_eval_segments_sdc.argtypes = [P, P, D, I, ctypes.POINTER(Segment), P, P, P, DP]
    lib.dtn_setup_dd.argtypes = [P, P, P, D, I]
    lib.shoot_eval_sdc.argtypes = [P, P, D, I, P, P, P, DP]
    lib.shoot_eval_sdc_dd.argtypes = [P, I, D, D, D, P, P, D, D, I, P, P, P, P, DP]
    lib.dtn_solve_multi_dd.argtypes = [P, P, P, I, P, P, P, P]
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.shoot_eval_batch.argtypes = [I, PP, PP, DP, ctypes.POINTER(ctypes.c_int), PP, PP, PP, DP]
    lib.shoot_eval_batch.restype = I
    lib.ww_profile.argtypes = [P, I]
    lib.ww_profile_read.argtypes = [P, I, DP, ctypes.POINTER(ctypes.c_int)]
    lib.ww_fallbacks.argtypes = [P, ctypes.POINTER(U)]
    lib.ww_thin_svd.argtypes = [P, P, I, I, DP, DP, P]
    lib.ww_levmar.argtypes = [P, DP, I, ctypes.POINTER(LmOpts), ctypes.POINTER(LmReport)]
    lib.ww_lm_default_opts.argtypes = [ctypes.POINTER(LmOpts)]
    lib.ww_bfgs.argtypes = [P, DP, I, ctypes.POINTER(BfgsOpts), ctypes.POINTER(BfgsReport)]
    lib.ww_bfgs_default_opts.argtypes = [ctypes.POINTER(BfgsOpts)]
    lib.ww_last_error.restype = ctypes.c_char_p
    lib.ww_version.restype = ctypes.c_char_p
    for name in ["ww_create", "ww_set_stream", "ww_set_tableau", "dtn_setup", "dtn_solve_multi",
                 "dtn_solve_multi_noalloc",
                 "shoot_setup", "shoot_eval", "shoot_adjoint", "ww_profile", "ww_profile_read", "ww_fallbacks",
                 "ww_thin_svd", "ww_levmar", "ww_lm_default_opts", "ww_bfgs", "ww_bfgs_default_opts"]:
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise WWError(rc, _lib.ww_last_error().decode())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "need contiguous cuda float64"
    return ctypes.c_void_p(t.data_ptr())


def dop853():
    """Dormand-Prince 8(5,3) tableau, 12 stages of the 8th-order update, from SciPy's
    published coefficient table."""
    from scipy.integrate._ivp import dop853_coefficients as d
    s = d.N_STAGES
    return (np.ascontiguousarray(d.A[:s, :s], dtype=np.float64),
            np.ascontiguousarray(d.B, dtype=np.float64),
            np.ascontiguousarray(d.C[:s], dtype=np.float64))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Context:
    """One engine context on the current GPU, on torch's current stream.  strict=True
    disables the fallbacks (pivoted LU, FP64 after a failed refinement test): the
    calls then raise WW_EPIVOT / WW_EREFINE instead."""

    def __init__(self, n_max: int, r_max: int, mixed: bool = False, stream=None, tableau=None,
                 strict: bool = False, gmres: bool = False):
        self.lib = load()
        self.ptr = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s            # the library keeps the handle: keep the stream alive
        flags = (WW_MIXED if mixed else WW_FP64) | (WW_STRICT if strict else 0) | (WW_GMRES if gmres else 0)
        _check(self.lib.ww_create(ctypes.byref(self.ptr), n_max, r_max, flags,
                                  ctypes.c_void_p(s.cuda_stream)))
        self.n_max, self.r_max, self.mixed = n_max, r_max, mixed
        a, b, c = tableau if tableau is not None else dop853()
        self._tab = (a, b, c)
        _check(self.lib.ww_set_tableau(self.ptr, len(b), _dp(a), _dp(b), _dp(c)))
        self.N = None
        self.M = None

    def close(self):
        if self.ptr:
            self.lib.ww_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(self.lib.ww_set_stream(self.ptr, ctypes.c_void_p(stream.cuda_stream)))
        self._stream = stream

    def _keep(self, t: torch.Tensor):
        """A temporary read by stream-ordered work on the context's stream must not be
        reused by torch's allocator before that work has run."""
        if self._stream != torch.cuda.current_stream(t.device):
            t.record_stream(self._stream)
        return t

    # ----- DtN -----
    def dtn_setup(self, surface: torch.Tensor, h: float, tau: float = 0.0):
        N = surface.numel()
        _check(self.lib.dtn_setup(self.ptr, _ptr(surface), float(h), float(tau), N))
        self.dN = N

    def dtn_solve_multi(self, rhs: torch.Tensor, want_mu: bool = False, noalloc: bool = False):
        """rhs: (N, nrhs) column-major -> pass as a (nrhs, N) contiguous tensor transposed.
        Accepts a (N,) vector or an (N, nrhs) tensor; returns tensors of the same shape.
        noalloc=True calls dtn_solve_multi_noalloc (work arrays in the library's fixed
        per-GPU workspace; the outputs are still allocated here)."""
        vec = rhs.dim() == 1
        cols = rhs.reshape(-1, 1) if vec else rhs
        N, nrhs = cols.shape
        cm = self._keep(cols.t().contiguous())         # column-major storage
        out = torch.empty_like(cm)
        mu = torch.empty_like(cm) if want_mu else None
        fn = self.lib.dtn_solve_multi_noalloc if noalloc else self.lib.dtn_solve_multi
        _check(fn(self.ptr, _ptr(cm), nrhs, _ptr(out), _ptr(mu)))
        o = out.t()
        m = mu.t() if want_mu else None
        if vec:
            o = o.reshape(-1)
            m = m.reshape(-1) if want_mu else None
        return (o, m) if want_mu else o

    # ----- shooting -----
    def shoot_setup(self, N, h, tau, g, basis: torch.Tensor, q_fixed: torch.Tensor | None = None):
        """basis: (2N, M) tensor (column k = eta part; phi part)."""
        M = basis.shape[1]
        bcm = self._keep(basis.t().contiguous())
        qf = self._keep(q_fixed.contiguous()) if q_fixed is not None else None
        _check(self.lib.shoot_setup(self.ptr, N, float(h), float(tau), float(g), _ptr(bcm), _ptr(qf), M))
        self.N, self.M = N, M

    def shoot_eval(self, params: torch.Tensor, T: float, nsteps: int, jacobian: bool = True,
                   drdT: bool = True):
        if self.N is None:      # let the library report WW_ENOSETUP
            _check(self.lib.shoot_eval(self.ptr, _ptr(params.contiguous()), float(T), int(nsteps),
                                       _ptr(params), None, None, None))
        N, M = self.N, self.M
        dev = params.device
        r = torch.empty(N, dtype=torch.float64, device=dev)
        Jc = torch.empty((M, N), dtype=torch.float64, device=dev) if jacobian else None
        d = torch.empty(N, dtype=torch.float64, device=dev) if drdT else None
        f = ctypes.c_double(0.0)
        _check(self.lib.shoot_eval(self.ptr, _ptr(params.contiguous()), float(T), int(nsteps),
                                   _ptr(r), _ptr(Jc), _ptr(d), ctypes.byref(f)))
        return dict(r=r, J=Jc.t() if jacobian else None, drdT=d, f=f.value)

    def shoot_eval_sdc(self, params: torch.Tensor, T: float, nsteps: int, jacobian: bool = True,
                       drdT: bool = True):
        """shoot_eval marched with SDC15 (shoot_eval_sdc)."""
        N, M = self.N, self.M
        dev = params.device
        r = torch.empty(N, dtype=torch.float64, device=dev)
        Jc = torch.empty((M, N), dtype=torch.float64, device=dev) if jacobian else None
        d = torch.empty(N, dtype=torch.float64, device=dev) if drdT else None
        f = ctypes.c_double(0.0)
        _check(self.lib.shoot_eval_sdc(self.ptr, _ptr(params.contiguous()), float(T), int(nsteps),
                                       _ptr(r), _ptr(Jc), _ptr(d), ctypes.byref(f)))
        return dict(r=r, J=Jc.t() if jacobian else None, drdT=d, f=f.value)

    def shoot_eval_sdc_dd(self, N: int, h: float, tau: float, g: float, q0_hi: torch.Tensor,
                          q0_lo: torch.Tensor | None, T: float, nsteps: int, T_lo: float = 0.0,
                          drdT: bool = True):
        """The base march in double-double with SDC15 (shoot_eval_sdc_dd).  q0 = [eta | phi]
        as hi (and lo) planes of 2N; returns r and dr/dT as (hi, lo) pairs of device
        tensors and f as (hi, lo) floats."""
        dev = q0_hi.device
        e = lambda: torch.empty(N, dtype=torch.float64, device=dev)
        rh, rl = e(), e()
        dh, dl = (e(), e()) if drdT else (None, None)
        f = (ctypes.c_double * 2)()
        _check(self.lib.shoot_eval_sdc_dd(self.ptr, int(N), float(h), float(tau), float(g),
                                          _ptr(q0_hi.contiguous()),
                                          _ptr(q0_lo.contiguous()) if q0_lo is not None else None,
                                          float(T), float(T_lo), int(nsteps), _ptr(rh), _ptr(rl), _ptr(dh),
                                          _ptr(dl), f))
        return dict(r=(rh, rl), drdT=(dh, dl) if drdT else None, f=(f[0], f[1]))

    def shoot_eval_segments_sdc(self, params: torch.Tensor, T: float, segments, jacobian: bool = True,
                                drdT: bool = True):
        """shoot_eval_segments with SDC15 steps (shoot_eval_segments_sdc)."""
        return self.shoot_eval_segments(params, T, segments, jacobian, drdT, _fn=self.lib.shoot_eval_segments_sdc)

    def shoot_eval_segments(self, params: torch.Tensor, T: float, segments, jacobian: bool = True,
                            drdT: bool = True, _fn=None):
        """The march over time segments on non-uniform meshes (shoot_eval_segments).
        segments: dicts with N, nsteps, theta, rho and refine_at (REFINE_PI default);
        the outputs live on the last segment's grid."""
        segs = (Segment * len(segments))(*[Segment(int(q["N"]), int(q["nsteps"]), float(q["theta"]),
                                                   float(q["rho"]), int(q.get("refine_at", REFINE_PI)))
                                           for q in segments])
        N, M = int(segments[-1]["N"]), (self.M if self.M is not None else 0)
        dev = params.device
        r = torch.empty(N, dtype=torch.float64, device=dev)
        Jc = torch.empty((M, N), dtype=torch.float64, device=dev) if jacobian else None
        d = torch.empty(N, dtype=torch.float64, device=dev) if drdT else None
        f = ctypes.c_double(0.0)
        fn = _fn if _fn is not None else self.lib.shoot_eval_segments
        _check(fn(self.ptr, _ptr(params.contiguous()), float(T), len(segments), segs, _ptr(r), _ptr(Jc), _ptr(d),
                  ctypes.byref(f)))
        return dict(r=r, J=Jc.t() if jacobian else None, drdT=d, f=f.value)

    def dtn_setup_dd(self, surface_hi: torch.Tensor, surface_lo: torch.Tensor | None, h: float):
        """Double-double DtN set-up (dtn_setup_dd): surface = hi + lo planes."""
        hi = self._keep(surface_hi.contiguous())
        lo = self._keep(surface_lo.contiguous()) if surface_lo is not None else None
        _check(self.lib.dtn_setup_dd(self.ptr, _ptr(hi), _ptr(lo), float(h), int(hi.shape[0])))
        self.dN = int(hi.shape[0])

    def dtn_solve_multi_dd(self, rhs_hi: torch.Tensor, rhs_lo: torch.Tensor | None, want_mu: bool = False):
        """G psi in double-double for rhs (N, nrhs) given as hi and lo planes: returns
        (out_hi, out_lo) or (out_hi, out_lo, mu_hi, mu_lo)."""
        N, R = rhs_hi.shape
        hi = self._keep(rhs_hi.t().contiguous())
        lo = self._keep(rhs_lo.t().contiguous()) if rhs_lo is not None else None
        mk = lambda: torch.empty((R, N), dtype=torch.float64, device=rhs_hi.device)
        oh, ol = mk(), mk()
        mh, ml = (mk(), mk()) if want_mu else (None, None)
        _check(self.lib.dtn_solve_multi_dd(self.ptr, _ptr(hi), _ptr(lo), R, _ptr(oh), _ptr(ol), _ptr(mh), _ptr(ml)))
        out = (oh.t(), ol.t())
        return out + (mh.t(), ml.t()) if want_mu else out

    def fallbacks(self) -> int:
        """WW_FB_* bits behind the results of the last call on this context."""
        b = ctypes.c_uint(0)
        _check(self.lib.ww_fallbacks(self.ptr, ctypes.byref(b)))
        return b.value

    def thin_svd(self, A: torch.Tensor, want_u: bool = False):
        """A: (N, n) tensor (column-major storage is made here).  Returns (sigma, V, U):
        sigma (n,) descending and V (n, n) as NumPy arrays, U (N, n) on the device or None."""
        N, n = A.shape
        cm = self._keep(A.t().contiguous())
        sig = np.zeros(n)
        V = np.zeros((n, n), order="F")
        U = torch.empty((n, N), dtype=torch.float64, device=A.device) if want_u else None
        _check(self.lib.ww_thin_svd(self.ptr, _ptr(cm), N, n, _dp(sig), _dp(V), _ptr(U)))
        return sig, V, (U.t() if want_u else None)

    def levmar(self, c0, nsteps: int, opts: dict | None = None, hist_cap: int = 0):
        """Levenberg-Marquardt with delayed Jacobian updates on the shooting problem of
        shoot_setup.  c0 = (T, params...).  Returns dict(c, f, delta, evals_r, evals_J,
        reason, history) -- history rows (c_new, f_new, accepted) of the tried steps."""
        n = self.M + 1
        c = np.ascontiguousarray(np.array(c0, dtype=np.float64))
        assert c.shape == (n,)
        o = LmOpts()
        _check(self.lib.ww_lm_default_opts(ctypes.byref(o)))
        for k, v in (opts or {}).items():
            setattr(o, k, v)
        h = np.zeros((max(hist_cap, 1), n + 2))
        rep = LmReport()
        rep.history = _dp(h) if hist_cap > 0 else None
        rep.hist_cap = hist_cap
        _check(self.lib.ww_levmar(self.ptr, _dp(c), int(nsteps), ctypes.byref(o), ctypes.byref(rep)))
        return dict(c=c, f=rep.f, delta=rep.delta, evals_r=rep.evals_r, evals_J=rep.evals_J,
                    reason=LM_REASONS.get(rep.reason, rep.reason),
                    history=h[:min(rep.n_hist, hist_cap)] if hist_cap > 0 else None)

    def bfgs(self, c0, nsteps: int, opts: dict | None = None, hist_cap: int = 0):
        """BFGS with the adjoint gradient (Sec. 3.2) on the shooting problem of
        shoot_setup.  c0 = (T, params...).  Returns dict(c, f, gnorm, iters, evals,
        reason, history) -- history rows (c, f) after every iteration."""
        n = self.M + 1
        c = np.ascontiguousarray(np.array(c0, dtype=np.float64))
        assert c.shape == (n,)
        o = BfgsOpts()
        _check(self.lib.ww_bfgs_default_opts(ctypes.byref(o)))
        for k, v in (opts or {}).items():
            setattr(o, k, v)
        h = np.zeros((max(hist_cap, 1), n + 1))
        rep = BfgsReport()
        rep.history = _dp(h) if hist_cap > 0 else None
        rep.hist_cap = hist_cap
        _check(self.lib.ww_bfgs(self.ptr, _dp(c), int(nsteps), ctypes.byref(o), ctypes.byref(rep)))
        return dict(c=c, f=rep.f, gnorm=rep.gnorm, iters=rep.iters, evals=rep.evals,
                    reason=BFGS_REASONS.get(rep.reason, rep.reason),
                    history=h[:min(rep.n_hist, hist_cap)] if hist_cap > 0 else None)

    def tuning(self) -> dict:
        """The context's launch and scheduling choices (ww_get_tuning)."""
        t = Tuning()
        _check(self.lib.ww_get_tuning(self.ptr, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **choices):
        """Change some of the launch and scheduling choices (ww_set_tuning; the others
        keep their current values)."""
        cur = self.tuning()
        unknown = set(choices) - set(cur)
        if unknown:
            raise ValueError(f"unknown tuning fields {sorted(unknown)}")
        cur.update(choices)
        t = Tuning(**{k: int(v) for k, v in cur.items()})
        _check(self.lib.ww_set_tuning(self.ptr, ctypes.byref(t)))

    def profile(self, enable: bool = True, kernel_events: bool = False):
        """Timestamps around the phases of every stage; with kernel_events, also HIP
        events around every block-LU step launched outside a graph (phase 4)."""
        _check(self.lib.ww_profile(self.ptr, (1 if enable else 0) | (2 if enable and kernel_events else 0)))

    def profile_read(self, phase: int) -> float:
        """Mean duration (ms) of a phase over every stage of every step replayed since
        the last profile(True): 0 block LU, 1 base chain, 2 column chain."""
        return self.profile_stats(phase)[0]

    def profile_stats(self, phase: int):
        """(mean duration in ms, number of intervals) of a phase since the last
        profile(True)."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int(0)
        _check(self.lib.ww_profile_read(self.ptr, phase, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def shoot_adjoint(self, params: torch.Tensor, T: float, nsteps: int, ckpt_every: int = 16):
        M = self.M
        grad = torch.empty(M, dtype=torch.float64, device=params.device)
        dfdT = ctypes.c_double(0.0)
        f = ctypes.c_double(0.0)
        _check(self.lib.shoot_adjoint(self.ptr, _ptr(params.contiguous()), float(T), int(nsteps),
                                      int(ckpt_every), _ptr(grad), ctypes.byref(dfdT), ctypes.byref(f)))
        return dict(grad=grad, dfdT=dfdT.value, f=f.value)


def shoot(ctx: Context, params: torch.Tensor, T: float, nsteps: int, jacobian: bool = True):
    """(r, J, drdT, f) of one shoot_eval: r = phi(T/4)/sqrt(N), J its Jacobian in the
    parameters (None when jacobian=False), drdT = dr/dT, f = r.r/2."""
    out = ctx.shoot_eval(params, T, nsteps, jacobian=jacobian, drdT=True)
    return out["r"], out["J"], out["drdT"], out["f"]


def to_dev(a, device="cuda") -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


def shoot_eval_batch(contexts, params, T, nsteps, jacobian=True, drdT=True):
    """Batched shoot_eval over distinct contexts (one instance each).  Returns a list of
    dicts like Context.shoot_eval."""
    lib = load()
    n = len(contexts)
    VP = ctypes.c_void_p * n
    outs = []
    rp, Jp, dp = VP(), VP(), VP()
    for i, (c, p) in enumerate(zip(contexts, params)):
        N, M = c.N, c.M
        r = torch.empty(N, dtype=torch.float64, device=p.device)
        Jc = torch.empty((M, N), dtype=torch.float64, device=p.device) if jacobian else None
        d = torch.empty(N, dtype=torch.float64, device=p.device) if drdT else None
        outs.append((r, Jc, d))
        rp[i] = r.data_ptr()
        Jp[i] = Jc.data_ptr() if jacobian else None
        dp[i] = d.data_ptr() if drdT else None
    cp = VP(*[c.ptr.value for c in contexts])
    pc = [p.contiguous() for p in params]   # held until the call has synchronised
    pp = VP(*[p.data_ptr() for p in pc])
    Ta = (ctypes.c_double * n)(*[float(t) for t in T])
    Na = (ctypes.c_int * n)(*[int(k) for k in nsteps])
    fa = (ctypes.c_double * n)()
    _check(lib.shoot_eval_batch(n, cp, pp, Ta, Na, rp, Jp if jacobian else None,
                                dp if drdT else None, fa))
    return [dict(r=r, J=Jc.t() if Jc is not None else None, drdT=d, f=fa[i])
            for i, (r, Jc, d) in enumerate(outs)]
