"""Batched form: instances of uneven N, depth, tension, M and step count, run
interleaved by shoot_eval_batch, give exactly the results of separate shoot_eval calls,
and match the oracle."""
import math

import numpy as np
import pytest

from oracle import ww_oracle as O
from paper_1210_5672_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ww():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5672_amd import ww
    return ww, torch


def _instances():
    rng = np.random.default_rng(77)
    specs = [(64, math.inf, 0.0, 6, 12), (96, 0.8, 0.01, 9, 20), (128, 2.0, 0.0, 3, 8), (64, 0.3, 0.005, 4, 16)]
    out = []
    for n, (N, h, tau, M, nsteps) in enumerate(specs):
        p = np.zeros(M)
        p[0] = 0.03 if math.isinf(h) else min(0.03, 0.2 * h)
        p[1:] = rng.normal(0, 1e-3, M - 1)
        out.append(W.Workload(f"b{n}", N, h, tau, 1.0, M, W.linear_period(h, tau), nsteps, p,
                              W.cosine_basis(N, M), np.zeros(2 * N)))
    return out


def test_batch_equals_separate_runs_and_oracle():
    ww, torch = _ww()
    ws = _instances()
    ctxs, params = [], []
    for w in ws:
        s = torch.cuda.Stream()
        c = ww.Context(n_max=max(64, w.N), r_max=w.M + 1, stream=s)
        c.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        ctxs.append(c)
        params.append(ww.to_dev(w.params))
    print("batch of", len(ws), flush=True)
    torch.cuda.synchronize()
    outb = ww.shoot_eval_batch(ctxs, params, [w.T for w in ws], [w.nsteps for w in ws])
    torch.cuda.synchronize()
    for w, c, p, ob in zip(ws, ctxs, params, outb):
        one = c.shoot_eval(p, w.T, w.nsteps)
        torch.cuda.synchronize()
        for k in ("r", "J", "drdT"):
            assert torch.equal(ob[k], one[k]), (w.name, k)
        assert ob["f"] == one["f"]
        ref = O.shoot_eval(w.N, w.h, w.tau, w.g, w.basis, w.q_fixed, w.params, w.T, w.nsteps)
        er = np.linalg.norm(ob["r"].cpu().numpy() - ref["r"]) / np.linalg.norm(ref["r"])
        eJ = np.linalg.norm(ob["J"].cpu().numpy() - ref["J"]) / np.linalg.norm(ref["J"])
        print(w.name, er, eJ)
        assert er < 1e-12 and eJ < 1e-12


def test_batch_rejects_repeated_context():
    ww, torch = _ww()
    w = _instances()[0]
    c = ww.Context(n_max=64, r_max=w.M + 1)
    c.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
    p = ww.to_dev(w.params)
    with pytest.raises(ww.WWError) as ei:
        ww.shoot_eval_batch([c, c], [p, p], [w.T, w.T], [2, 2])
    assert ei.value.name == "WW_EINVAL"


def test_batch_non_contiguous_params_and_shoot_tuple():
    """Parameter views that are not contiguous are copied and kept alive for the call;
    ww.shoot returns (r, J, drdT, f) of shoot_eval."""
    ww, torch = _ww()
    ws = _instances()[:2]
    ctxs, views, plain = [], [], []
    for w in ws:
        c = ww.Context(n_max=max(64, w.N), r_max=w.M + 1, stream=torch.cuda.Stream())
        c.shoot_setup(w.N, w.h, w.tau, w.g, ww.to_dev(w.basis), ww.to_dev(w.q_fixed))
        ctxs.append(c)
        pd = ww.to_dev(w.params)
        views.append(torch.stack([pd, pd], dim=1)[:, 0])   # stride 2
        plain.append(pd)
    assert not views[0].is_contiguous()
    torch.cuda.synchronize()
    ov = ww.shoot_eval_batch(ctxs, views, [w.T for w in ws], [w.nsteps for w in ws])
    op = ww.shoot_eval_batch(ctxs, plain, [w.T for w in ws], [w.nsteps for w in ws])
    torch.cuda.synchronize()
    for a, b in zip(ov, op):
        for k in ("r", "J", "drdT"):
            assert torch.equal(a[k], b[k])
    r, J, drdT, f = ww.shoot(ctxs[0], plain[0], ws[0].T, ws[0].nsteps)
    torch.cuda.synchronize()
    assert torch.equal(r, op[0]["r"]) and torch.equal(J, op[0]["J"]) and f == op[0]["f"]
