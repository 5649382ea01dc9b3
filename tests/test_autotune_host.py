"""Autotuner logic (choice, margin, on-disk cache) with a stand-in context, and
the library's validation of launch-shape settings (host only, no GPU)."""
import json

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from paper_1503_08462_amd import autotune
from workloads import configs


class FakeOpts:
    precision = ae.PREC_MIXED
    smoother = ae.SMOOTH_CHEBYSHEV


class FakeCtx:
    """Three levels, width 16; timings from a table, every call recorded."""

    def __init__(self, times):
        self.times = times  # (kind, level, cpt) -> us
        self.opts = FakeOpts()
        self.set = {}
        self.calls = []

    def info(self):
        return {"qe": 16, "levels": 3, "dims": np.array([1000, 400, 100])}

    def level_nnz(self, level):
        return [7000, 3000, 900][level]

    def set_cpt(self, kind, level, cpt):
        self.set[(kind, level)] = cpt

    def get_cpt(self, kind, level):
        c = self.set.get((kind, level), 0)
        return c if c else 2  # a stand-in built-in choice

    def tune_time(self, kind, level, cpt, reps):
        self.calls.append((kind, level, cpt))
        return self.times.get((kind, level, cpt), 10.0)


def test_picks_fastest_beyond_margin_and_caches(tmp_path):
    times = {(0, 0, 4): 7.0, (0, 0, 8): 8.0,   # clearly faster: taken
             (0, 1, 4): 9.9,                   # within the 3 % margin: built-in kept
             (1, 1, 8): 5.0}
    ctx = FakeCtx(times)
    path = str(tmp_path / "t.json")
    rep = autotune.tune(ctx, cache_path=path, reps=3)
    assert ctx.set[(0, 0)] == 4
    assert ctx.set[(0, 1)] == 2
    assert ctx.set[(1, 1)] == 8
    assert ctx.set[(1, 0)] == 2
    # groups: levels 0 and 1 (the coarsest has no row kernels), wide kind from level 1
    assert sorted((v["kind"], v["level"]) for v in rep.values()) == [
        ("fp64", 0), ("fp64", 1), ("fp64_wide", 1), ("vcycle", 0), ("vcycle", 1)]
    widths = {k.split("|")[-1] for k in rep}
    assert widths == {"w16", "w32"}
    stored = json.load(open(path))
    assert len(stored) == 5
    # second context of the same shape: no timing, same choices
    ctx2 = FakeCtx({})
    autotune.tune(ctx2, cache_path=path)
    assert ctx2.calls == []
    assert ctx2.set == ctx.set


def test_candidates_respect_width():
    assert autotune.candidates(16) == [2, 4, 8]
    assert autotune.candidates(4) == [2, 4]
    assert autotune.candidates(68) == [2, 4]
    assert autotune.candidates(136) == [4, 8]  # 136 / 2 = 68 lanes would exceed a wavefront


def test_library_validates_launch_shape():
    p = configs.config(0)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=130))
    assert ctx.get_cpt(ae.TUNE_VCYCLE, 0) == 4  # width 4: the built-in rule takes 4 columns per lane
    ctx.set_cpt(ae.TUNE_VCYCLE, 0, 2)
    assert ctx.get_cpt(ae.TUNE_VCYCLE, 0) == 2
    ctx.set_cpt(ae.TUNE_VCYCLE, 0, 0)
    assert ctx.get_cpt(ae.TUNE_VCYCLE, 0) == 4
    for bad in (1, 3, 8, 16):  # 8 does not divide width 4
        with pytest.raises(ae.AmgEigError) as e:
            ctx.set_cpt(ae.TUNE_VCYCLE, 0, bad)
        assert e.value.code == ae.EINVAL
    with pytest.raises(ae.AmgEigError):
        ctx.set_cpt(3, 0, 2)
    with pytest.raises(ae.AmgEigError):
        ctx.set_cpt(ae.TUNE_FP64, 99, 2)
    us = __import__("ctypes").c_double()
    rc = ae._lib.amg_eig_tune_time(ctx._c, ae.TUNE_VCYCLE, 0, 2, 1, __import__("ctypes").byref(us))
    assert rc == ae.ESTATE  # not bound
    ctx.close()
