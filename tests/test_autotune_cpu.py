"""Host logic of the autotuner (paper_1210_5672_amd/autotune.py): the JSON cache and
the coordinate descent, with a scripted cost in place of timed marches."""
import json

from paper_1210_5672_amd import autotune as A


def test_cache_roundtrip_and_lookup(tmp_path):
    p = str(tmp_path / "cache.json")
    assert A.load(p) == {}
    k = A.key(1024, 128, False, arch="gfx950")
    assert k == "gfx950/N1024/M128/fp64"
    assert A.key(512, 40, True, arch="gfx950", batch=True) == "gfx950/N512/M40/mixed/batch"
    assert A.key(1024, 200, False, arch="gfx950", segments=True) == "gfx950/N1024/M200/fp64/segments"
    t = {"lag": 8, "lu_group": 2, "lu_streams": 3, "graph_parts": 10, "minv_wgs": 256, "blu_strip": 4,
         "dtn_rows": 8, "gemm_split": 4, "asm_cw": 16, "gemm_rows": 32, "lag_fp32": 0}
    A.store(k, t, 0.0123, "test", p)
    data = json.load(open(p))
    assert data[k]["tuning"] == t and data[k]["seconds"] == 0.0123
    assert A.lookup(1024, 128, False, p, arch="gfx950") == t
    assert A.lookup(1024, 128, True, p, arch="gfx950") is None
    # a second entry keeps the first
    A.store(A.key(256, 64, False, arch="gfx950"), dict(t, lag=6), 0.002, "test", p)
    assert A.lookup(1024, 128, False, p, arch="gfx950") == t


def test_descent_finds_the_separable_optimum():
    """A cost that is a sum of one term per choice (plus a rejected region): the descent
    reaches the best candidate of every choice and never keeps a rejected one."""
    best_of = {n: vals[-1] for n, vals in A.SPACE.items()}
    start = {n: vals[0] for n, vals in A.SPACE.items()}

    def measure(ch):
        if ch["lag"] == 6:            # e.g. a lag too short: the march falls back
            return None
        return 1.0 + sum(0.0 if ch[n] == best_of[n] else 0.1 for n in ch)

    best, t, hist = A.descend(measure, start, list(A.SPACE), passes=3, log=lambda *a: None)
    expect = dict(best_of)
    if expect["lag"] == 6:
        expect["lag"] = start["lag"]
    for n in A.SPACE:
        if n == "lag" and best_of["lag"] == 6:
            assert best["lag"] != 6
        else:
            assert best[n] == expect[n], n
    assert all(m is None or m >= t for _, m in hist)


def test_defaults_of_the_library_are_candidates():
    """The first candidate of every choice is ww_create's default, so that a cache entry
    is never worse than no tuning at all (the descent starts from the defaults)."""
    defaults = {"lag": 8, "lu_group": 2, "lu_streams": 3, "graph_parts": 10, "minv_wgs": 1 << 20,
                "blu_strip": 4, "dtn_rows": 8, "gemm_split": 4, "asm_cw": 16,
                 "gemm_rows": 32, "lag_fp32": 0, "lag_sweeps": 2}
    assert set(defaults) == set(A.SPACE)
    for n, v in defaults.items():
        assert A.SPACE[n][0] == v, n
