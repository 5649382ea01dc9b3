"""GPU parity of the multicolour Gauss-Seidel smoother (the paper's smoother of
Section 4.1, rows visited colour by colour) against the oracle's "mcgs"
V-cycle: each correction from the same random start step by step, then the
converged pairs.  Tolerances as in the other parity tests: 1e-10 relative per
eigenvalue in FP64 (per step: the wanted ones; the extra ones of a wide block
5e-9), 1e-5 per step and 1e-6 converged in mixed precision, eigenspaces
<= 1e-6 by the sine of the largest principal angle."""
import numpy as np
import pytest

import paper_1503_08462_amd as ae
from workloads import configs, prng
from tests.helpers import compare_subspaces, reference_eigenvalues
from tests.test_gpu_parity import _say, _torch, gpu_state, make_ctx, oracle_for, oracle_solve

pytestmark = pytest.mark.gpu

# (name, problem, coarse_max, explicit q_e or 0).  lshape24j: 4 colours on the
# finest level, the V-cycle below it in the dense tail; cube12: up to ~30
# colours on coarse Galerkin levels with rows of more than 64 entries per
# wavefront; osc96_qe16: a finest level and a level 1 above the tail, so the
# prolongation reads a Gauss-Seidel result from a level below; lshape40j_qe36:
# a block wider than 32 columns.
CASES = [
    ("lshape24j", lambda: configs.lshape(24, q=6, jitter_seed=5), 150, 0),
    ("cube12", lambda: configs.cube(12, q=32), 150, 0),  # the whole 32-member low cluster
    ("osc96_qe16", lambda: configs.oscillator(96, q=10), 200, 16),
    ("lshape40j_qe36", lambda: configs.lshape(40, q=10, jitter_seed=3), 300, 36),
]


@pytest.mark.parametrize("name,make,cm,qe", CASES)
@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED])
def test_gauss_seidel_step_parity_and_solve(name, make, cm, qe, prec):
    _torch()
    p = make()
    _say("%s multicolour Gauss-Seidel prec=%d" % (name, prec))
    kw = dict(coarse_max=cm, precision=prec, smoother=ae.SMOOTH_GAUSS_SEIDEL)
    if qe:
        kw["qe"] = qe
    ctx = make_ctx(p, **kw)
    o, A, M = oracle_for(p, ctx, smoother="mcgs", explicit_qe=qe > 0)
    q, qe = p["q"], ctx.info()["qe"]
    for l in range(ctx.info()["levels"] - 1):
        assert np.array_equal(ctx.colouring(l)[0], o.levels[l].colour)
    ctx.init(ae.INIT_RANDOM, seed=11)
    lam_o, U_o = o.random_start(prng.random_block(11, p["n"], qe))
    # FP64: the wanted Ritz values to 1e-10 after every step; the extra ones at
    # the top of a wide block to 5e-9.  The small eigensolver stops its
    # Rayleigh-quotient iteration at a residual of 1e-8 |rho|, which leaves a
    # Ritz value an error of order residual^2 / gap; early in a solve the last
    # Ritz value of the 36-wide block has a neighbour in the projected pencil
    # close enough for that to reach 9e-10, with Chebyshev smoothing too.
    if prec == ae.PREC_FP64:
        want_tol, all_tol = 1e-10, 5e-9
    else:
        want_tol = all_tol = 1e-5
    for step in range(3):
        ctx.correct(1)
        th, U, pr = gpu_state(ctx)
        lam_o, U_o = o.correction(0, lam_o, U_o)
        err = np.abs(th / lam_o - 1)
        print("step %d: max relative difference %.2e (wanted %.2e)" % (step + 1, err.max(), err[:q].max()))
        assert err[:q].max() < want_tol and err.max() < all_tol, (step, th, lam_o)
    lam, ok = ctx.solve(tol=1e-10, max_steps=300)
    th, U, pr = gpu_state(ctx)
    assert ok, pr
    assert ctx.info()["qe"] == qe
    print("GPU: %d corrections" % pr["steps"])
    lo, Uo = oracle_solve(o, 1e-11)
    err = np.abs(lam / lo[:q] - 1)
    print("max relative eigenvalue difference %.2e" % err.max())
    assert np.all(err < (1e-10 if prec == ae.PREC_FP64 else 1e-6))
    worst, ms = compare_subspaces(reference_eigenvalues(p, qe + 1), Uo, U, M, q, qe=qe)
    print("compared prefixes", ms, "largest sine %.2e" % worst)
    assert worst < 1e-6
    assert np.abs(U.T @ (M @ U) - np.eye(qe)).max() < 1e-11
    assert o.residuals(0, th, U)[:q].max() <= 1e-10 * 1.01
    ctx.close()


def test_gauss_seidel_graph_replay_equals_eager():
    """The colour sweeps captured in a hipGraph: every replay, with host reads
    between them, equals the eager step bit for bit."""
    torch = _torch()
    p = configs.oscillator(96, q=6)
    _say("multicolour Gauss-Seidel graph replay vs eager")
    res = {0: [], 1: []}
    for g in (0, 1):
        s = torch.cuda.Stream()
        ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"],
                         ae.defaults(coarse_max=200, use_graph=g, precision=ae.PREC_MIXED,
                                     smoother=ae.SMOOTH_GAUSS_SEIDEL))
        ctx.bind(stream=s)
        ctx.init(ae.INIT_NESTED)
        for _ in range(4):
            ctx.correct(1)
            th, U, _ = gpu_state(ctx)
            res[g].append((th.copy(), U.copy()))
        ctx.close()
    for (te, Ue), (tg, Ug) in zip(res[0], res[1]):
        assert np.array_equal(te, tg) and np.array_equal(Ue, Ug)
