"""Serving form on the GPU: requests of uneven size admitted under a memory
budget and advanced together on several streams give exactly the eigenvalues
each request gets when it is solved alone.  The block width is fixed (qe = 8):
the automatic width control acts on progress reports, whose cadence differs
between a served request and a solo solve."""
import sys

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from paper_1503_08462_amd.serving import Server
from workloads import configs

pytestmark = pytest.mark.gpu


def test_served_requests_equal_solo_solves():
    import torch
    assert torch.cuda.is_available()
    print("[case] serving 5 requests, 3 streams", flush=True)
    sys.stdout.flush()
    probs = [configs.square(16, q=4), configs.lshape(16, q=4, jitter_seed=3), configs.oscillator(40, q=6),
             configs.lshape(24, q=4, jitter_seed=4), configs.square(48, q=5)]
    opts = ae.defaults(coarse_max=100, qe=8, precision=ae.PREC_FP64)
    tol = 1e-9
    fps = sorted(ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], opts).footprint() for p in probs)
    srv = Server(fps[-1] + fps[-2], n_streams=3, steps_per_round=2, opts=opts)
    ids = [srv.submit(p, tol=tol, max_steps=300) for p in probs]
    res = srv.run()
    assert srv.peak_in_use <= srv.budget
    for rid, p in zip(ids, probs):
        solo_opts = ae.defaults(coarse_max=100, qe=8, precision=ae.PREC_FP64, tol=tol)
        ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], solo_opts)
        ctx.bind()
        lam, ok = ctx.solve(tol=tol, max_steps=300)
        assert ok, (rid, "solo")
        assert res[rid]["converged"], (rid, "served", res[rid]["steps"])
        assert np.array_equal(lam, res[rid]["lam"]), (rid, lam, res[rid]["lam"])
        ctx.close()
    lat = srv.latency()
    assert lat["count"] == len(probs) and lat["p50_s"] > 0


def test_served_with_joint_starts_and_per_stream_steps_equal_solo():
    """The other serving options: requests admitted together start jointly
    (init_batch_joint), and the corrections run with one stream per request and
    no joint stage (correct_batch); each result equals its solo solve."""
    import torch
    assert torch.cuda.is_available()
    print("[case] serving 4 requests, joint starts, per-stream steps", flush=True)
    sys.stdout.flush()
    probs = [configs.square(16, q=4), configs.lshape(16, q=4, jitter_seed=3), configs.oscillator(40, q=6),
             configs.lshape(24, q=4, jitter_seed=4)]
    opts = ae.defaults(coarse_max=100, qe=8, precision=ae.PREC_FP64)
    tol = 1e-9
    srv = Server(1 << 34, n_streams=2, steps_per_round=3, opts=opts,
                 init_fn=lambda cs: ae.init_batch_joint(cs),
                 batch_fn=lambda cs, steps: ae.correct_batch(cs, steps))
    ids = [srv.submit(p, tol=tol, max_steps=300) for p in probs]
    res = srv.run()
    for rid, p in zip(ids, probs):
        ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"],
                         ae.defaults(coarse_max=100, qe=8, precision=ae.PREC_FP64, tol=tol))
        ctx.bind()
        lam, ok = ctx.solve(tol=tol, max_steps=300)
        assert ok, (rid, "solo")
        assert res[rid]["converged"], (rid, "served", res[rid]["steps"])
        assert np.array_equal(lam, res[rid]["lam"]), (rid, lam, res[rid]["lam"])
        ctx.close()
