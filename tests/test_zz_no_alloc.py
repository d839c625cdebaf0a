"""The allocation-free DtN solve (dtn_solve_multi_noalloc, for callers that cannot
allocate device memory) against the allocating entry point dtn_solve_multi on the same
context: two calls in a row, the second with fewer right-hand sides; both precision
forms; a padded grid; and the size limit of its fixed workspace."""
import numpy as np
import pytest

from paper_1210_5672_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("N,h", [(1024, 0.5), (96, 0.7)])
def test_noalloc_solve_matches_dtn_solve_multi(N, h, mixed):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5672_amd import ww
    print(f"noalloc N={N} h={h} mixed={mixed}", flush=True)
    ctx = ww.Context(n_max=N, r_max=129, mixed=mixed)
    ctx.dtn_setup(ww.to_dev(W.random_surface(N, seed=7, amp=0.04)), h)
    for call, nrhs in enumerate((129, 17)):
        rhs = ww.to_dev(W.random_rhs(N, nrhs, seed=11 + call))
        ref, ref_mu = ctx.dtn_solve_multi(rhs, want_mu=True)
        torch.cuda.synchronize()
        free0, res0 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
        out, mu = ctx.dtn_solve_multi(rhs, want_mu=True, noalloc=True)
        out2 = ctx.dtn_solve_multi(rhs, noalloc=True)
        torch.cuda.synchronize()
        free1, res1 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
        e = (_rel(out, ref), _rel(mu, ref_mu), _rel(out2, ref))
        # device memory taken during the two calls, apart from what torch's allocator
        # reserved for the caller's output tensors: the library allocates nothing
        taken = (free0 - free1) - (res1 - res0)
        print(f"  call {call} nrhs={nrhs}: rel diff out {e[0]:.2e} mu {e[1]:.2e} again {e[2]:.2e}; "
              f"device memory taken outside torch {taken / 2**20:.1f} MiB", flush=True)
        assert max(e) < TOL, e
        assert taken < (2 << 20), taken


def test_noalloc_solve_rejects_sizes_beyond_its_workspace():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5672_amd import ww
    N, nrhs = 2048, 300          # 7 * 2048 * 300 doubles = 34.4 MB > 32 MiB
    print("noalloc size limit", flush=True)
    ctx = ww.Context(n_max=N, r_max=nrhs)
    ctx.dtn_setup(ww.to_dev(W.random_surface(N, seed=3, amp=0.03)), float("inf"))
    rhs = ww.to_dev(W.random_rhs(N, nrhs, seed=5))
    with pytest.raises(ww.WWError) as ei:
        ctx.dtn_solve_multi(rhs, noalloc=True)
    assert ei.value.name == "WW_EINVAL" and "fixed workspace" in str(ei.value)
    # within the limit on the same context: matches the allocating entry point
    small = ww.to_dev(W.random_rhs(N, 292, seed=6))
    e = _rel(ctx.dtn_solve_multi(small, noalloc=True), ctx.dtn_solve_multi(small))
    print(f"  N=2048 nrhs=292: rel diff {e:.2e}", flush=True)
    assert e < TOL
