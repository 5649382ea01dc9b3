"""Launch-shape tuning on the GPU: every columns-per-lane choice, and the
autotuner's, give bit-identical solves; the timings are positive."""
import sys

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from paper_1503_08462_amd import autotune
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _solve(p, prec, qe, force=None, tune_path=None):
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"],
                     ae.defaults(coarse_max=200, qe=qe, precision=prec))
    ctx.bind()
    rep = None
    if tune_path is not None:
        rep = autotune.tune(ctx, cache_path=tune_path, reps=3)
    if force is not None:
        nl = ctx.info()["levels"]
        for level in range(nl - 1):
            for kind in (ae.TUNE_VCYCLE, ae.TUNE_FP64, ae.TUNE_FP64_WIDE):
                width = 2 * qe if kind == ae.TUNE_FP64_WIDE else qe
                if force in autotune.candidates(width) and not (kind == ae.TUNE_FP64_WIDE and level == 0):
                    ctx.set_cpt(kind, level, force)
    ctx.init(ae.INIT_NESTED)
    lam, ok = ctx.solve(1e-9, 300)
    pr = ctx.progress()
    ctx.close()
    return lam, ok, pr["steps"], rep


# q_e = 8 takes the narrow kernels; q_e = 40 the wide ones (the dual SpMM fused
# with the Gram products, whose pass of rows grows from 24 to 96 with the
# columns per lane while the Gram sums keep their order)
@pytest.mark.parametrize("qe", [8, 40])
@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED], ids=["fp64", "mixed"])
def test_launch_shape_does_not_change_results(prec, qe, tmp_path):
    p = configs.lshape(24, q=6, jitter_seed=2)
    _say("launch shapes, L-shape N=%d, qe=%d, prec=%d" % (p["n"], qe, prec))
    ref, ok, steps, _ = _solve(p, prec, qe)
    assert ok
    for cpt in (2, 4, 8):
        _say("forced cpt %d" % cpt)
        lam, ok2, steps2, _ = _solve(p, prec, qe, force=cpt)
        assert ok2 and steps2 == steps
        assert np.array_equal(lam, ref), (cpt, lam - ref)
    _say("autotuned")
    lam, ok3, steps3, rep = _solve(p, prec, qe, tune_path=str(tmp_path / "cpt.json"))
    assert ok3 and steps3 == steps and np.array_equal(lam, ref)
    assert rep and all(v["us"] is None or min(v["us"].values()) > 0 for v in rep.values())
    # a second context of the same shape takes the cached choices without timing
    lam, _, _, rep2 = _solve(p, prec, qe, tune_path=str(tmp_path / "cpt.json"))
    assert all(v["us"] is None for v in rep2.values())
    assert {k: v["cpt"] for k, v in rep2.items()} == {k: v["cpt"] for k, v in rep.items()}
    assert np.array_equal(lam, ref)
