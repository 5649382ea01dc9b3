"""GPU parity of corrections with m > 1 AMG cycles on the linear equation
(Algorithm 3.1, eq. (3.2)): after the first V-cycle, each further cycle starts
from the previous iterate with the residual of the linear equation at it.  From
the same random start every correction agrees with the oracle's m-cycle
correction step by step, with and without the shift of Remark 3.1 and under
each smoother; the converged pairs agree with the oracle and an independent
reference, and more cycles take fewer corrections."""
import numpy as np
import pytest

import paper_1503_08462_amd as ae
from oracle import Oracle
from workloads import configs, prng
from tests.helpers import compare_subspaces, mats, reference_eigenvalues
from tests.test_gpu_parity import _say, _torch, gpu_state, make_ctx, oracle_solve

pytestmark = pytest.mark.gpu

CASES = [
    # (name, problem, coarse_max, q_e, smoother, oracle smoother, m, shift)
    ("square31_cheb_m2", lambda: configs.config(0), 130, 4, ae.SMOOTH_CHEBYSHEV, "chebyshev", 2, 0.0),
    ("osc48_cheb_m3_shift", lambda: configs.oscillator(48, q=10), 150, 16, ae.SMOOTH_CHEBYSHEV, "chebyshev", 3, 1.8),
    ("lshape16j_gs_m2", lambda: configs.lshape(16, q=6, jitter_seed=4), 150, 8, ae.SMOOTH_GAUSS_SEIDEL, "mcgs", 2, 0.0),
    ("osc32_l1_m2", lambda: configs.oscillator(32, q=6), 120, 8, ae.SMOOTH_L1JACOBI, "l1jacobi", 2, 0.0),
]


@pytest.mark.parametrize("name,make,cm,qe,sm,osm,m,shift", CASES, ids=[c[0] for c in CASES])
def test_m_cycle_correction_matches_oracle(name, make, cm, qe, sm, osm, m, shift):
    _torch()
    p = make()
    q = p["q"]
    A, M = mats(p)
    cmin = 2 * (2 * q + 8) + 2
    _say("%s: m = %d, shift %g" % (name, m, shift))
    ctx = make_ctx(p, coarse_max=cm, coarse_min=cmin, qe=qe, smoother=sm, shift=shift, vcycles=m)
    o = Oracle(A, M, q=q, qe=qe, coarse_max=cm, coarse_min=cmin, smoother=osm, shift=shift, cycles=m)
    assert [L.n for L in o.levels] == ctx.info()["dims"].tolist()
    ctx.init(ae.INIT_RANDOM, seed=3)
    lam_o, U_o = o.random_start(prng.random_block(3, p["n"], qe))
    for step in range(3):
        ctx.correct(1)
        th, U, pr = gpu_state(ctx)
        lam_o, U_o = o.correction(0, lam_o, U_o)
        err = np.abs(th / lam_o - 1)
        print("step %d: max relative difference %.2e (wanted %.2e)" % (step + 1, err.max(), err[:q].max()))
        assert err[:q].max() < 1e-10 and err.max() < 5e-9, (step, th, lam_o)
    lam, ok = ctx.solve(tol=1e-10, max_steps=300)
    th, U, pr = gpu_state(ctx)
    assert ok, pr
    lo, Uo = oracle_solve(o, 1e-11)
    err = np.abs(lam / lo[:q] - 1)
    print("GPU: %d corrections, max relative eigenvalue difference %.2e" % (pr["steps"], err.max()))
    assert np.all(err < 1e-10)
    worst, ms = compare_subspaces(reference_eigenvalues(p, qe + 1), Uo, U, M, q, qe=qe)
    print("compared prefixes", ms, "largest sine %.2e" % worst)
    assert worst < 1e-6
    assert np.abs(U.T @ (M @ U) - np.eye(qe)).max() < 1e-11
    ctx.close()


def test_more_cycles_fewer_corrections_mixed():
    """Mixed precision (FP32 cycles under the FP64 residual): one, two and
    three cycles per correction converge to the same eigenvalues, in fewer
    corrections as m grows."""
    torch = _torch()
    p = configs.lshape(48, q=8, jitter_seed=2)
    q = p["q"]
    ref = reference_eigenvalues(p, q)
    steps = []
    for m in (1, 2, 3):
        ctx = make_ctx(p, coarse_max=300, qe=12, precision=ae.PREC_MIXED, vcycles=m)
        lam, ok = ctx.solve(tol=1e-9, max_steps=300)
        torch.cuda.synchronize()
        assert ok
        steps.append(ctx.progress()["steps"])
        assert np.abs(lam / ref - 1).max() < 1e-9
        ctx.close()
    _say("mixed lshape48j: corrections for m = 1, 2, 3: %s" % steps)
    assert steps[1] < steps[0] and steps[2] <= steps[1]


def test_vcycles_out_of_range_refused():
    p = configs.config(0)
    for m in (0, 17):
        with pytest.raises(ae.AmgEigError) as e:
            ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(vcycles=m))
        assert e.value.code == ae.EINVAL


def test_m_cycles_graph_and_joint_equal_eager_solo():
    """With m = 2 cycles a captured step replays the eager step bit for bit, and
    a joint batch of two requests on two streams (amg_eig_correct_batch_joint)
    gives bitwise the iterates of the same requests corrected one by one."""
    torch = _torch()
    probs = [(configs.lshape(24, q=6, jitter_seed=4), dict(coarse_max=200, qe=8, precision=ae.PREC_MIXED)),
             (configs.oscillator(40, q=6), dict(coarse_max=150, qe=8, precision=ae.PREC_FP64))]

    def ctx_for(p, kw, graph, stream):
        c = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(use_graph=graph, vcycles=2, **kw))
        c.bind(stream=stream)
        c.init(ae.INIT_NESTED)
        return c

    def state(c):
        qe = c.info()["qe"]
        return c.progress()["theta"].copy(), c.iterate().cpu().numpy()[:, :qe].copy()

    _say("m = 2: eager, captured and joint steps")
    eager = [ctx_for(p, kw, 0, torch.cuda.Stream()) for p, kw in probs]
    graph = [ctx_for(p, kw, 1, torch.cuda.Stream()) for p, kw in probs]
    joint = [ctx_for(p, kw, 0, torch.cuda.Stream()) for p, kw in probs]
    for c in eager + graph:
        c.correct(4)
    ae.correct_batch_joint(joint, 4)
    torch.cuda.synchronize()
    for e, g, j in zip(eager, graph, joint):
        te, ue = state(e)
        tg, ug = state(g)
        tj, uj = state(j)
        assert np.array_equal(te, tg) and np.array_equal(ue, ug)
        assert np.array_equal(te, tj) and np.array_equal(ue, uj)
    for c in eager + graph + joint:
        c.close()
