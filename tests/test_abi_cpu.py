"""Host-only checks of the C ABI: the library loads and exports every entry point
declared in include/ww.h; argument errors are reported without touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ww.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def _lib():
    from paper_1210_5672_amd import ww
    if not os.path.exists(ww.LIB_PATH):
        pytest.skip("library not built")
    return ww, ww.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["ww_create", "ww_destroy", "ww_set_tableau", "dtn_setup", "dtn_solve_multi",
              "shoot_setup", "shoot_eval", "shoot_adjoint", "ww_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    ww, lib = _lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) <= set(ww.EXPORTS)


def test_argument_errors_without_gpu():
    ww, lib = _lib()
    a = (ctypes.c_double * 4)()
    assert lib.ww_set_tableau(None, 2, a, a, a) == -1
    assert b"null" in lib.ww_last_error()
    assert lib.dtn_setup(None, None, 1.0, 0.0, 64) == -1
    assert lib.dtn_solve_multi(None, None, 1, None, None) == -1
    assert lib.shoot_setup(None, 64, 1.0, 0.0, 1.0, None, None, 4) == -1
    assert lib.shoot_eval(None, None, 1.0, 1, None, None, None, None) == -1
    assert lib.shoot_adjoint(None, None, 1.0, 1, 16, None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.ww_create(None, 64, 4, 0, None) == -1
    assert lib.ww_create(ctypes.byref(out), 70, 4, 0, None) == -1      # 70 is not 2^a 3^b
    assert lib.ww_create(ctypes.byref(out), 4096, 4, 0, None) == -1    # above 2048
    assert lib.ww_create(ctypes.byref(out), 64, 4, 8, None) == -1      # unknown flag
    assert lib.ww_fallbacks(None, None) == -1
    assert lib.ww_levmar(None, None, 1, None, None) == -1
    assert lib.ww_thin_svd(None, None, 4, 2, None, None, None) == -1


def test_levenberg_marquardt_defaults_are_the_papers():
    """App. C: f_tol = 1e-26, g_tol = 1e-13, max_stepsJ = 10, df_tol = 1e-5 (host only)."""
    ww, lib = _lib()
    o = ww.LmOpts()
    assert lib.ww_lm_default_opts(ctypes.byref(o)) == 0
    assert (o.f_tol, o.g_tol, o.df_tol, o.max_steps_J) == (1e-26, 1e-13, 1e-5, 10)


def test_bfgs_defaults():
    ww, lib = _lib()
    o = ww.BfgsOpts()
    assert lib.ww_bfgs_default_opts(ctypes.byref(o)) == 0
    assert (o.f_tol, o.g_tol, o.ckpt_every) == (1e-26, 1e-13, 16)
    assert lib.ww_bfgs(None, None, 1, None, None) == -1


def test_jacobi_round_schedule_covers_every_pair_once():
    """The circle-method pairing of the one-sided Jacobi SVD (round rd, pair q: players
    rd and n2 - 1 for q = 0, else (rd + q) and (rd - q) mod (n2 - 1)) visits every pair of
    the n columns exactly once per sweep and never a column twice in one round (the
    pairs of a round run in parallel); players >= n are padding."""
    for n in (1, 2, 3, 8, 33, 129, 257):
        n2 = (n + 1) & ~1
        m = n2 - 1
        seen = {}
        for rd in range(max(m, 0)):
            used = set()
            for q in range(n2 // 2):
                a = rd if q == 0 else (rd + q) % m
                b = m if q == 0 else (rd - q + m) % m
                a, b = min(a, b), max(a, b)
                assert a != b
                assert a not in used and b not in used
                used.update((a, b))
                if b < n:
                    seen[(a, b)] = seen.get((a, b), 0) + 1
        assert len(seen) == n * (n - 1) // 2 and all(v == 1 for v in seen.values()), n


def test_fallback_decision_table():
    """The redo a march takes from its status bits (host logic, no GPU): a small pivot
    (1, 8) redoes pivoted (also FP64; every stage then uses its own factors);
    unconverged lagged-factor (32) or GMRES (64) solves are redone on each stage's own
    factors, also when the surface crossed the bed (16), since that state came from
    the unconverged solves; a crossing on those factors, or without such solves, is
    reported (its small pivots too); a failed mixed refinement test redoes in FP64;
    WW_STRICT contexts never redo."""
    ww, lib = _lib()
    F = lib.ww_next_fallback
    PIV, FP64, DIRECT, STRICT = ww.WW_FB_PIVOTED, ww.WW_FB_FP64, ww.WW_FB_DIRECT, ww.WW_STRICT
    assert F(0, 0, 0) == 0
    assert F(0, 0, 32) == DIRECT and F(0, 0, 64) == DIRECT
    assert F(0, 0, 32 | 16) == DIRECT            # crossing on lagged factors: redo first
    assert F(0, 0, 64 | 16 | 2) == DIRECT
    assert F(0, DIRECT, 32 | 16) == 0           # crossing on the direct factors: report
    assert F(0, 0, 16) == 0 and F(0, 0, 16 | 1) == 0
    assert F(0, 0, 1) == PIV | FP64 and F(0, 0, 8) == PIV | FP64
    assert F(0, PIV | FP64, 8) == 0              # the pivoted factors failed too: report
    assert F(0, DIRECT, 1 | 32) == PIV | FP64
    assert F(0, 0, 1 | 32) == PIV | FP64         # pivots first: it also ends the lagging
    assert F(0, 0, 1 | 32 | 16) == PIV | FP64
    assert F(0, PIV | FP64, 32) == DIRECT
    assert F(ww.WW_MIXED, 0, 4) == FP64 and F(ww.WW_MIXED, FP64, 4) == 0
    assert F(0, 0, 2) == 0                       # non-finite state: report
    for st in (1, 4, 8, 16, 32, 64, 32 | 16):
        assert F(STRICT, 0, st) == 0
        assert F(STRICT | ww.WW_MIXED, 0, st) == 0


def test_noalloc_solve_rejects_bad_arguments_without_gpu():
    ww, lib = _lib()
    assert lib.dtn_solve_multi_noalloc(None, None, 1, None, None) == -1
    assert b"null" in lib.ww_last_error()


def test_tuning_calls_reject_null_arguments_without_gpu():
    ww, lib = _lib()
    t = ww.Tuning()
    assert lib.ww_get_tuning(None, ctypes.byref(t)) == -1   # WW_EINVAL
    assert lib.ww_set_tuning(None, ctypes.byref(t)) == -1


def test_blu_step_flop_count_is_the_lu_count():
    """The per-launch flop figure of the block-LU step: summed over the steps, the left
    factors and the trailing updates of a right-looking block LU come to
    2/3 (N^3 - N b^2), i.e. 2/3 N^3 less the work of the diagonal-block inversions;
    brute-force count over the tiles at small sizes."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for N, b in ((64, 64), (256, 64), (1024, 64), (96, 8)):
        nb = N // b
        brute = 0
        for k in range(nb - 1):
            for i in range(k + 1, nb):
                brute += 2 * b ** 3          # L_ik = A_ik D_k
                for j in range(k + 1, nb):
                    brute += 2 * b ** 3      # A_ij -= L_ik A_kj
        assert bench.blu_step_flops(N, b) == brute
        assert abs(brute - (2.0 / 3.0) * (N ** 3 - N * b * b)) < 1e-6 * N ** 3
