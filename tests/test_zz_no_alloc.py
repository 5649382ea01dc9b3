"""The bind that allocates nothing (the library's static device workspace)
against the regular bind into a caller's workspace, through the C ABI: two
binds in a row on one device, the second with a smaller problem, each solve
equal bit for bit to the same solve in a caller workspace (same kernels and
launch shapes); the first context loses the workspace to the second; a
problem whose footprint exceeds the static workspace is refused."""
import sys

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _solve(ctx, p, torch, tol=1e-9):
    U = torch.zeros((p["n"], p["q"]), dtype=torch.float64, device="cuda")
    lam, ok = ctx.solve(tol=tol, max_steps=300, U_out=U)
    torch.cuda.synchronize()
    assert ok
    return lam, U.cpu().numpy()


def test_static_bind_equals_caller_workspace_bind():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    probs = [configs.lshape(40, q=6, jitter_seed=3), configs.square(24, q=4)]  # the second is smaller
    held = []
    for p in probs:
        kw = dict(coarse_max=200, qe=8, precision=ae.PREC_MIXED)
        a = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(**kw))
        _say("static bind, N=%d, footprint %d bytes" % (p["n"], a.footprint()))
        a.bind_static()
        assert a._ws_bytes == 64 << 20 and a.footprint() <= a._ws_bytes
        lam_a, U_a = _solve(a, p, torch)
        b = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(**kw))
        b.bind()
        lam_b, U_b = _solve(b, p, torch)
        assert np.array_equal(lam_a, lam_b) and np.array_equal(U_a, U_b)
        b.close()
        held.append(a)
    # the first context lost the static workspace to the second
    with pytest.raises(ae.AmgEigError) as e:
        held[0].solve(tol=1e-9, max_steps=10)
    assert e.value.code == ae.ESTATE
    for a in held:
        a.close()


def test_static_bind_refuses_a_footprint_beyond_its_size():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p = configs.lshape(160, q=10, jitter_seed=2)
    a = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(qe=16))
    _say("static bind refused, N=%d, footprint %d bytes" % (p["n"], a.footprint()))
    assert a.footprint() > 64 << 20
    with pytest.raises(ae.AmgEigError) as e:
        a.bind_static()
    assert e.value.code == ae.EWORKSPACE
    a.close()
