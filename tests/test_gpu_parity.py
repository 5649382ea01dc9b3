"""GPU parity of the HIP solve phase against the FP64 CPU oracle.

Every case prints its name before touching the GPU.  Tolerances: eigenvalues
1e-10 relative (FP64 mode) / 1e-6 (mixed mode), eigenspaces by the sine of the
largest principal angle (M inner product) <= 1e-6 over gap-delimited prefixes.
"""
import sys

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from oracle import Oracle
from workloads import configs, prng
from tests.helpers import brute_force, compare_subspaces, mats

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def gpu_state(ctx):
    pr = ctx.progress()
    qe = ctx.info()["qe"]
    U = ctx.iterate().cpu().numpy()[:, :qe].copy()
    return pr["theta"], U, pr


def make_ctx(p, **kw):
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(**kw))
    ctx.bind()
    return ctx


def oracle_for(p, ctx, smoother="chebyshev"):
    A, M = mats(p)
    info = ctx.info()
    o = Oracle(A, M, q=p["q"], qe=info["qe"], coarse_max=ctx.opts.coarse_max,
               coarse_min=ctx.opts.coarse_min if ctx.opts.coarse_min > 0 else 2 * (2 * p["q"] + 8) + 2,
               smoother=smoother)
    assert [L.n for L in o.levels] == info["dims"].tolist()
    return o, A, M


def test_random_start_and_step_parity_config0():
    """Config 0 (N = 961, q = 4, seed 1): the device start block is the same
    SplitMix64 stream the oracle draws; Rayleigh-Ritz of the start and each of
    the first corrections agree step by step."""
    _torch()
    p = configs.config(0)
    _say("config0 random start, step parity, FP64")
    ctx = make_ctx(p, coarse_max=130, smoother=ae.SMOOTH_L1JACOBI)
    o, A, M = oracle_for(p, ctx, smoother="l1jacobi")
    qe = ctx.info()["qe"]
    ctx.init(ae.INIT_RANDOM, seed=1)
    th, U, _ = gpu_state(ctx)
    U0 = prng.random_block(1, p["n"], qe)
    lam_o, U_o = o.random_start(U0)
    assert np.abs(th / lam_o - 1).max() < 1e-11
    assert compare_subspaces(lam_o, U_o, U, M, qe - 1) < 1e-8
    for step in range(3):
        ctx.correct(1)
        th, U, pr = gpu_state(ctx)
        lam_o, U_o = o.correction(0, lam_o, U_o)
        assert pr["steps"] == step + 1
        assert np.abs(th / lam_o - 1).max() < 1e-10, (step, th, lam_o)
        assert compare_subspaces(lam_o, U_o, U, M, qe - 1) < 1e-7
    lam, ok = ctx.solve(tol=1e-10, max_steps=200)
    assert ok
    ref, Uref = brute_force(p, qe + 1)
    th, U, pr = gpu_state(ctx)
    assert np.abs(lam / ref[:4] - 1).max() < 1e-10
    assert compare_subspaces(ref, Uref, U, M, 4) < 1e-6
    assert np.abs(U.T @ (M @ U) - np.eye(qe)).max() < 1e-12
    ctx.close()


SMALL = [
    ("lshape32j", lambda: configs.lshape(32, q=10, jitter_seed=2), 300),
    ("cube16", lambda: configs.cube(16, q=32), 400),  # the whole 32-member low cluster
    ("osc48", lambda: configs.oscillator(48, q=10), 200),
    ("quadrants16", lambda: configs.quadrants(16, q=6), 120),
    ("square63", lambda: configs.square(64, q=1), 150),
]


@pytest.mark.parametrize("name,make,cm", SMALL)
@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED])
def test_nested_solve_matches_oracle(name, make, cm, prec):
    _torch()
    p = make()
    _say("%s nested solve prec=%d" % (name, prec))
    ctx = make_ctx(p, coarse_max=cm, precision=prec)
    o, A, M = oracle_for(p, ctx)
    q, qe = p["q"], ctx.info()["qe"]
    lam, ok = ctx.solve(tol=1e-10, max_steps=300)
    th, U, pr = gpu_state(ctx)
    assert ok, pr
    lo, Uo, info = o.solve(tol=1e-11, max_steps=400)
    if prec == ae.PREC_FP64:
        # FP64 fixes lambda_j only to about eps * lambda_max / lambda_j
        kap = np.abs(A).sum(axis=1).max() / M.diagonal().min() / lo[:q]
        tol = np.maximum(1e-10, 10 * np.finfo(float).eps * kap)
    else:
        tol = 1e-6
    assert np.all(np.abs(lam / lo[:q] - 1) < tol)
    assert compare_subspaces(lo, Uo, U, M, q) < 1e-6
    assert np.abs(U.T @ (M @ U) - np.eye(qe)).max() < 1e-11
    # the device residuals agree with a CPU evaluation of the returned pairs
    rho_cpu = o.residuals(0, th, U)
    assert rho_cpu[:q].max() <= 1e-10 * 1.01
    ctx.close()


@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED])
def test_chebyshev_smoother_step_parity_and_solve(prec):
    """Degree-2 Chebyshev smoothing on [0.25, 1]: each correction agrees with
    the oracle's Chebyshev V-cycle step by step (FP64), and the converged pairs
    agree with the oracle's (both precisions) on a jittered L-shape."""
    _torch()
    p = configs.lshape(24, q=6, jitter_seed=5)
    _say("chebyshev smoother prec=%d" % prec)
    ctx = make_ctx(p, coarse_max=150, precision=prec, smoother=ae.SMOOTH_CHEBYSHEV, cheb_degree=2, cheb_lo=0.25)
    o, A, M = oracle_for(p, ctx, smoother="chebyshev")
    q, qe = p["q"], ctx.info()["qe"]
    ctx.init(ae.INIT_RANDOM, seed=11)
    lam_o, U_o = o.random_start(prng.random_block(11, p["n"], qe))
    for step in range(3):
        ctx.correct(1)
        th, U, pr = gpu_state(ctx)
        lam_o, U_o = o.correction(0, lam_o, U_o)
        tol = 1e-10 if prec == ae.PREC_FP64 else 1e-5
        assert np.abs(th / lam_o - 1).max() < tol, (step, th, lam_o)
    lam, ok = ctx.solve(tol=1e-10, max_steps=300)
    th, U, pr = gpu_state(ctx)
    assert ok, pr
    lo, Uo, info = o.solve(tol=1e-11, max_steps=400)
    assert np.abs(lam / lo[:q] - 1).max() < (1e-10 if prec == ae.PREC_FP64 else 1e-6)
    assert compare_subspaces(lo, Uo, U, M, q) < 1e-6
    assert o.residuals(0, th, U)[:q].max() <= 1e-10 * 1.01
    ctx.close()


WIDE = [
    # (name, problem, explicit q_e, precision): widths beyond one 16-column tile and
    # beyond 32 columns (the kernels' wide layouts)
    ("cube24_qe32", lambda: configs.cube(24, q=20), 32, ae.PREC_FP64),
    ("lshape40j_qe36", lambda: configs.lshape(40, q=10, jitter_seed=3), 36, ae.PREC_FP64),
    ("osc96_q64", lambda: configs.oscillator(96, q=64), 0, ae.PREC_MIXED),
]


@pytest.mark.parametrize("name,make,qe,prec", WIDE)
def test_wide_blocks_match_oracle(name, make, qe, prec):
    _torch()
    p = make()
    _say("%s wide block qe=%d prec=%d" % (name, qe, prec))
    ctx = make_ctx(p, qe=qe, precision=prec)
    o, A, M = oracle_for(p, ctx)
    q = p["q"]
    assert ctx.info()["qe"] == (qe if qe else o.qe)
    lam, ok = ctx.solve(tol=1e-9, max_steps=300)
    th, U, pr = gpu_state(ctx)
    assert ok, pr
    lo, Uo, info = o.solve(tol=1e-11, max_steps=400)
    if prec == ae.PREC_FP64:
        kap = np.abs(A).sum(axis=1).max() / M.diagonal().min() / lo[:q]
        tol = np.maximum(1e-10, 10 * np.finfo(float).eps * kap)
    else:
        tol = 1e-6
    assert np.all(np.abs(lam / lo[:q] - 1) < tol)
    assert compare_subspaces(lo, Uo, U, M, q) < 1e-6
    assert o.residuals(0, th, U)[:q].max() <= 1e-9 * 1.01
    ctx.close()


def test_user_start_equals_random_start():
    torch = _torch()
    p = configs.lshape(16, q=4, jitter_seed=3)
    _say("user start vs random start")
    a = make_ctx(p, coarse_max=100)
    qe = a.info()["qe"]
    a.init(ae.INIT_RANDOM, seed=9)
    a.correct(2)
    ta, Ua, _ = gpu_state(a)
    b = make_ctx(p, coarse_max=100)
    U0 = torch.tensor(prng.random_block(9, p["n"], qe), device="cuda", dtype=torch.float64)
    b.init(ae.INIT_USER, U=U0)
    b.correct(2)
    tb, Ub, _ = gpu_state(b)
    assert np.array_equal(ta, tb) and np.array_equal(Ua, Ub)
    a.close()
    b.close()


def test_bitwise_determinism():
    _torch()
    p = configs.oscillator(40, q=6)
    _say("determinism")
    outs = []
    for _ in range(2):
        ctx = make_ctx(p, coarse_max=150, precision=ae.PREC_MIXED)
        ctx.solve(tol=1e-9, max_steps=100)
        outs.append(gpu_state(ctx)[:2])
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_graph_replay_equals_eager():
    torch = _torch()
    p = configs.lshape(24, q=6, jitter_seed=4)
    _say("graph replay vs eager")
    res = []
    for g in (0, 1):
        s = torch.cuda.Stream()
        ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=200, use_graph=g))
        ctx.bind(stream=s)
        ctx.init(ae.INIT_NESTED)
        for _ in range(4):  # replays interleaved with host reads
            ctx.correct(1)
            th, U, pr = gpu_state(ctx)
            res.append((g, th.copy(), U.copy()))
        ctx.close()
    eager = [r for r in res if r[0] == 0]
    graph = [r for r in res if r[0] == 1]
    for e, gr in zip(eager, graph):
        assert np.array_equal(e[1], gr[1]) and np.array_equal(e[2], gr[2])


def test_config1_full_size_fp64_and_mixed():
    """Config 1 at full size (jittered L-shape, N = 195 585, q = 10)."""
    _torch()
    p = configs.config(1)
    A, M = mats(p)
    _say("config1 oracle")
    o = Oracle(A, M, q=10, qe=12, coarse_max=512, coarse_min=42, smoother="gs")
    lo, Uo, info = o.solve(tol=1e-10, max_steps=200)
    for prec in (ae.PREC_FP64, ae.PREC_MIXED):
        _say("config1 full size prec=%d" % prec)
        ctx = make_ctx(p, coarse_max=512, coarse_min=42, qe=12, precision=prec)
        lam, ok = ctx.solve(tol=1e-8, max_steps=300)
        th, U, pr = gpu_state(ctx)
        assert ok, pr
        assert pr["rho"][:10].max() <= 1e-8
        tol = 1e-10 if prec == ae.PREC_FP64 else 1e-6
        assert np.abs(lam / lo[:10] - 1).max() < tol
        assert compare_subspaces(lo, Uo, U, M, 10) < 1e-6
        rho_cpu = o.residuals(0, th, U)
        assert rho_cpu[:10].max() <= 1.01e-8
        ctx.close()
