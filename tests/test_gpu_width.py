"""Block width control of the solve driver on the GPU, through the C ABI.

The checkerboard cube has a cluster of 32 eigenvalues at the bottom of its
spectrum (one mode per kappa = 1 block, relative gaps below 0.6%, then a gap
of about 120%).  Its coarsest level spreads the cluster by tens of percent, so
the guard rule on the coarsest eigenvalues cuts it; with default options the
driver must then widen the block (the paper's extra eigenpairs, Section 4.5)
and still converge to the oracle's pairs.  Also: a solve with a tighter
tolerance after a converged one re-tests the iterate.
"""
import sys

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from oracle import Oracle
from workloads import configs
from tests.helpers import compare_subspaces, mats, reference_eigenvalues

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _state(ctx):
    pr = ctx.progress()
    qe = ctx.info()["qe"]
    return pr, ctx.iterate().cpu().numpy()[:, :qe].copy()


def _check_against_oracle(p, ctx, lam, prec, cm):
    """Oracle at the context's final width on its own hierarchy (same level
    sizes): eigenvalues, subspaces (the whole 32-member cluster), residuals."""
    A, M = mats(p)
    q = p["q"]
    info = ctx.info()
    qe = info["qe"]
    o = Oracle(A, M, q=q, qe=qe, coarse_max=cm, coarse_min=2 * (2 * q + 8) + 2, smoother="chebyshev")
    assert [L.n for L in o.levels] == info["dims"].tolist()
    lo, Uo, oi = o.solve(tol=1e-11, max_steps=400)
    assert oi["rho"][:q].max() <= 1e-11, oi["rho"][:q].max()
    pr, U = _state(ctx)
    err = np.abs(lam / lo[:q] - 1).max()
    print("width %d, max relative eigenvalue difference %.2e" % (qe, err))
    assert err < (1e-10 if prec == ae.PREC_FP64 else 1e-6)
    worst, ms = compare_subspaces(reference_eigenvalues(p, qe + 1), Uo, U, M, q, qe=qe)
    print("compared prefixes", ms, "largest sine %.2e" % worst)
    assert 32 in ms and worst < 1e-6
    assert o.residuals(0, pr["theta"], U)[:q].max() <= 1e-9 * 1.01


@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED], ids=["fp64", "mixed"])
def test_default_options_widen_a_cut_cluster_q6(prec):
    _torch()
    p = configs.cube(16, q=6)
    _say("cube16 q=6 default width prec=%d" % prec)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 6, ae.defaults(coarse_max=400, precision=prec))
    qe0 = ctx.info()["qe"]
    assert qe0 < 32  # the coarsest level cuts the cluster
    ctx.bind()
    lam, ok = ctx.solve(tol=1e-9, max_steps=300)
    assert ok, ctx.progress()
    print("width %d -> %d" % (qe0, ctx.info()["qe"]))
    assert ctx.info()["qe"] >= 32
    _check_against_oracle(p, ctx, lam, prec, 400)
    ctx.close()


def test_default_options_widen_then_narrow_q20():
    """q = 20: the coarse rule's block stalls inside the cluster, the doubled
    block converges, and the next start takes 32, the end of the cluster."""
    _torch()
    p = configs.cube(16, q=20)
    _say("cube16 q=20 default width, mixed")
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 20, ae.defaults(coarse_max=400, precision=ae.PREC_MIXED))
    qe0 = ctx.info()["qe"]
    assert qe0 < 32
    ctx.bind()
    lam, ok = ctx.solve(tol=1e-9, max_steps=300)
    assert ok, ctx.progress()
    wide = ctx.info()["qe"]
    print("width %d -> %d" % (qe0, wide))
    assert wide > 32
    _check_against_oracle(p, ctx, lam, ae.PREC_MIXED, 400)
    ctx.init(ae.INIT_NESTED)  # the converged wide block showed the cluster's end
    assert ctx.info()["qe"] == 32
    lam2, ok = ctx.solve(tol=1e-9, max_steps=300)
    assert ok and ctx.info()["qe"] == 32
    _check_against_oracle(p, ctx, lam2, ae.PREC_MIXED, 400)
    ctx.close()


def test_widening_inside_a_large_enough_workspace():
    """A workspace with room for the wider block: the driver widens in place
    (the matrices stay where they were uploaded) and the binding never
    rebinds; the result agrees with that of a context rebound for every
    widening."""
    torch = _torch()
    import ctypes
    p = configs.cube(16, q=6)
    _say("cube16 q=6 widening in place")
    a = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 6, ae.defaults(coarse_max=400, precision=ae.PREC_FP64))
    ws = torch.empty(8 * a.footprint(), dtype=torch.uint8, device="cuda")
    a.workspace = ws
    a.stream = torch.cuda.current_stream()
    rc = ae._lib.amg_eig_bind(a._c, ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(a.stream.cuda_stream))
    assert rc == ae.OK
    lam_a, ok = a.solve(tol=1e-9, max_steps=300)
    assert ok and a.workspace is ws and a.info()["qe"] >= 32
    b = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 6, ae.defaults(coarse_max=400, precision=ae.PREC_FP64))
    b.bind()
    lam_b, ok = b.solve(tol=1e-9, max_steps=300)
    assert ok and b.info()["qe"] == a.info()["qe"]
    assert np.abs(lam_a / lam_b - 1).max() < 1e-12
    a.close()
    b.close()


def test_tighter_tolerance_after_a_converged_solve():
    """solve(1e-6) then solve(1e-10) on the same context: the second call must
    re-test the converged iterate and continue to the tighter tolerance."""
    _torch()
    p = configs.lshape(24, q=6, jitter_seed=4)
    _say("solve 1e-6 then 1e-10")
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 6, ae.defaults(coarse_max=150))
    ctx.bind()
    _, ok = ctx.solve(tol=1e-6, max_steps=200)
    assert ok
    steps1 = ctx.progress()["steps"]
    lam, ok = ctx.solve(tol=1e-10, max_steps=200)
    pr, U = _state(ctx)
    assert ok and pr["steps"] > steps1
    A, M = mats(p)
    MU = M @ U[:, :6]
    R = A @ U[:, :6] - MU * pr["theta"][None, :6]
    rho = np.linalg.norm(R, axis=0) / (pr["theta"][:6] * np.linalg.norm(MU, axis=0))
    assert rho.max() <= 1e-10 * 1.01, rho
    ctx.close()


def test_narrowed_width_keeps_a_convergence_margin():
    """A jittered L-shape (N = 339 360, q = 32) whose coarse rule gives q_e = q:
    the block stalls (lambda_33 is only 1.8% above lambda_32), is widened, and
    converges.  The next start must not narrow back to a width whose first
    Ritz value past the block lies close to lambda_q (that block would
    contract by about (1 / 1.018)^2 per correction): both solves converge and
    the second keeps theta_{q_e+1} >= 1.25 theta_q inside the first's block."""
    _torch()
    r = configs.request_stream(32, seed=5, n_lo=10_000, n_hi=1_000_000)[24]
    p = configs.build_request(r)
    _say("L-shape N=%d q=%d, two solves with the default width control" % (p["n"], p["q"]))
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=512, tol=1e-8))
    ctx.bind()
    lam1, ok = ctx.solve(tol=1e-8, max_steps=400)
    assert ok
    wide = ctx.info()["qe"]
    th = ctx.progress()["theta"]
    ctx.init(ae.INIT_NESTED)
    lam2, ok = ctx.solve(tol=1e-8, max_steps=400)
    w = ctx.info()["qe"]
    print("widths %d then %d, %d corrections" % (wide, w, ctx.progress()["steps"]))
    assert ok and w <= wide
    if w < wide:
        assert th[w] >= 1.25 * th[p["q"] - 1]
    assert np.abs(lam2 / lam1 - 1).max() < 1e-9
    ctx.close()
