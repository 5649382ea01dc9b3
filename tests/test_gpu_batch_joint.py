"""Batching form with the small eigenproblems solved jointly: requests of uneven
N, q_e, precision and coarse dimension d_n, on shared and separate streams,
advanced by amg_eig_correct_batch_joint give bitwise the iterates and Ritz
values of the same requests corrected one by one (which the parity tests pin
to the oracle)."""
import sys

import numpy as np
import pytest

import paper_1503_08462_amd as ae
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


MEMBERS = [
    # (problem, options): uneven N, q_e, d_n and precision in one batch
    # (explicit widths: the width control acts on progress reports, whose
    # cadence differs between joint and separate runs)
    (lambda: configs.square(16, q=4), dict(coarse_max=100, qe=8, precision=ae.PREC_FP64)),
    (lambda: configs.lshape(24, q=6, jitter_seed=4), dict(coarse_max=200, qe=8, precision=ae.PREC_MIXED)),
    (lambda: configs.oscillator(40, q=6), dict(coarse_max=150, qe=8, precision=ae.PREC_FP64)),
    (lambda: configs.cube(12, q=20), dict(coarse_max=300, qe=36, precision=ae.PREC_FP64)),
    (lambda: configs.lshape(40, q=10, jitter_seed=3), dict(qe=12, precision=ae.PREC_MIXED)),
]


def _ctx(p, stream, **kw):
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(use_graph=0, **kw))
    ctx.bind(stream=stream)
    ctx.init(ae.INIT_NESTED)
    return ctx


def _state(ctx):
    qe = ctx.info()["qe"]
    return ctx.progress()["theta"].copy(), ctx.iterate().cpu().numpy()[:, :qe].copy()


def test_joint_steps_equal_separate_steps():
    torch = _torch()
    probs = [(make(), kw) for make, kw in MEMBERS]
    _say("joint batch of %d members, 3 streams, 3 + 2 steps" % len(probs))
    streams = [torch.cuda.Stream() for _ in range(3)]
    joint = [_ctx(p, streams[i % 3], **kw) for i, (p, kw) in enumerate(probs)]
    solo = [_ctx(p, torch.cuda.Stream(), **kw) for p, kw in probs]
    for steps in (3, 2):
        ae.correct_batch_joint(joint, steps)
        for c in solo:
            c.correct(steps)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(joint, solo)):
            ta, Ua = _state(a)
            tb, Ub = _state(b)
            assert np.array_equal(ta, tb), (i, ta, tb)
            assert np.array_equal(Ua, Ub), i
    for c in joint + solo:
        c.close()


def test_joint_solve_with_members_converging_at_different_steps():
    torch = _torch()
    probs = [(make(), kw) for make, kw in MEMBERS[:3]]
    _say("joint batch until every member converges")
    s = torch.cuda.Stream()
    tol = 1e-9
    joint = [_ctx(p, s, tol=tol, **kw) for p, kw in probs]
    done = [False] * len(joint)
    for _ in range(100):
        ae.correct_batch_joint(joint, 2)
        done = [c.progress()["converged"] for c in joint]
        if all(done):
            break
    assert all(done)
    for (p, kw), c in zip(probs, joint):
        ref = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(use_graph=0, tol=tol, **kw))
        ref.bind()
        lam, ok = ref.solve(tol=tol, max_steps=300)
        assert ok
        assert np.array_equal(c.progress()["theta"][:p["q"]], lam)
        ref.close()
        c.close()


def test_joint_batch_beyond_one_launch_table():
    """More members than one launch table holds (64): the batch is split over
    several launches and every member still matches its separate run."""
    torch = _torch()
    n = 67
    _say("joint batch of %d members, one stream" % n)
    probs = [configs.square(10 + (i % 4), q=2 + (i % 3)) for i in range(n)]
    s = torch.cuda.Stream()
    joint = [_ctx(p, s, coarse_max=60, precision=ae.PREC_FP64) for p in probs]
    ae.correct_batch_joint(joint, 2)
    for i, p in enumerate(probs):
        ref = _ctx(p, s, coarse_max=60, precision=ae.PREC_FP64)
        ref.correct(2)
        ta, Ua = _state(joint[i])
        tb, Ub = _state(ref)
        assert np.array_equal(ta, tb) and np.array_equal(Ua, Ub), i
        ref.close()
    for c in joint:
        c.close()


def test_joint_batch_rejects_bad_lists():
    torch = _torch()
    _say("joint batch argument checks")
    p = configs.square(12, q=2)
    c = _ctx(p, torch.cuda.Stream(), coarse_max=60)
    with pytest.raises(ae.AmgEigError):
        ae.correct_batch_joint([c, c], 1)
    u = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=60))
    u.bind()
    with pytest.raises(ae.AmgEigError):
        ae.correct_batch_joint([c, u], 1)  # u is bound but not initialised
    ae.correct_batch_joint([], 1)
    c.close()
    u.close()


def test_joint_graph_parts_equal_eager_joint():
    """Members that replay their own parts from captured graphs (replays
    interleaved with host reads) match members launched eagerly, bitwise."""
    torch = _torch()
    probs = [(make(), kw) for make, kw in MEMBERS[:4]]
    _say("joint batch, graph parts vs eager parts, 4 members, 2 streams")
    res = {}
    for g in (0, 1):
        streams = [torch.cuda.Stream() for _ in range(2)]
        cs = []
        for i, (p, kw) in enumerate(probs):
            ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(use_graph=g, **kw))
            ctx.bind(stream=streams[i % 2])
            ctx.init(ae.INIT_NESTED)
            cs.append(ctx)
        res[g] = []
        for _ in range(4):
            ae.correct_batch_joint(cs, 1)
            res[g].append([_state(c) for c in cs])
        for c in cs:
            c.close()
    for e_round, g_round in zip(res[0], res[1]):
        for (te, Ue), (tg, Ug) in zip(e_round, g_round):
            assert np.array_equal(te, tg) and np.array_equal(Ue, Ug)


def test_joint_nested_start_equals_separate_starts():
    """Members with different numbers of levels started together (the small
    eigenproblems of each level in shared launches) hold bitwise the block and
    Ritz values of separate nested starts, before and after joint steps."""
    torch = _torch()
    probs = [(make(), kw) for make, kw in MEMBERS]
    _say("joint nested start of %d members, 2 streams" % len(probs))
    streams = [torch.cuda.Stream() for _ in range(2)]
    joint = []
    for i, (p, kw) in enumerate(probs):
        ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(use_graph=0, **kw))
        ctx.bind(stream=streams[i % 2])
        joint.append(ctx)
    assert len({len(c.info()["dims"]) for c in joint}) > 1  # uneven hierarchies
    ae.init_batch_joint(joint)
    solo = [_ctx(p, torch.cuda.Stream(), **kw) for p, kw in probs]
    for a, b in zip(joint, solo):
        ta, Ua = _state(a)
        tb, Ub = _state(b)
        assert np.array_equal(ta, tb) and np.array_equal(Ua, Ub)
        assert a.progress()["steps"] == 0
    ae.correct_batch_joint(joint, 2)
    for c in solo:
        c.correct(2)
    for a, b in zip(joint, solo):
        ta, Ua = _state(a)
        tb, Ub = _state(b)
        assert np.array_equal(ta, tb) and np.array_equal(Ua, Ub)
    for c in joint + solo:
        c.close()
