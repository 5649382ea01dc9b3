"""GPU parity of the shifted correction equation (Remark 3.1): the V-cycle of
A_k - sigma M_k on every level, the coarsest solve with A_n - sigma M_n.  Each
correction from the same random start agrees with the oracle's shifted
correction step by step (the same sigma on both sides), and the converged
pairs with the oracle's and an independent reference.  Tolerances as in the
other parity tests."""
import numpy as np
import pytest

import paper_1503_08462_amd as ae
from oracle import Oracle
from workloads import configs, prng
from tests.helpers import compare_subspaces, mats, reference_eigenvalues
from tests.test_gpu_parity import _say, _torch, gpu_state, make_ctx, oracle_for, oracle_solve

pytestmark = pytest.mark.gpu

CASES = [
    # (name, problem, coarse_max, q_e, smoother, oracle smoother)
    ("osc64_cheb", lambda: configs.oscillator(64, q=10), 150, 16, ae.SMOOTH_CHEBYSHEV, "chebyshev"),
    ("lshape32j_gs", lambda: configs.lshape(32, q=6, jitter_seed=2), 200, 8, ae.SMOOTH_GAUSS_SEIDEL, "mcgs"),
    ("cube12_l1", lambda: configs.cube(12, q=32), 150, 44, ae.SMOOTH_L1JACOBI, "l1jacobi"),
]


@pytest.mark.parametrize("name,make,cm,qe,sm,osm", CASES)
@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED])
def test_shifted_correction_matches_oracle(name, make, cm, qe, sm, osm, prec):
    _torch()
    p = make()
    q = p["q"]
    A, M = mats(p)
    # sigma = 0.9 lambda_1 of the coarsest level of the unshifted hierarchy
    probe = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], q, ae.defaults(coarse_max=cm))
    sigma = 0.9 * float(probe.coarse_eigenvalues()[0])
    probe.close()
    _say("%s shift %.6g prec=%d" % (name, sigma, prec))
    cmin = 2 * (2 * q + 8) + 2
    kw = dict(coarse_max=cm, coarse_min=cmin, precision=prec, smoother=sm, shift=sigma)
    if qe:
        kw["qe"] = qe
    ctx = make_ctx(p, **kw)
    # the width the context chose (checked against the oracle's rule), then the
    # shifted oracle on the same hierarchy
    qe = oracle_for(p, ctx, smoother=osm, explicit_qe=qe > 0)[0].qe
    o = Oracle(A, M, q=q, qe=qe, coarse_max=cm, coarse_min=cmin, smoother=osm, shift=sigma)
    assert [L.n for L in o.levels] == ctx.info()["dims"].tolist()
    qe = ctx.info()["qe"]
    ctx.init(ae.INIT_RANDOM, seed=5)
    lam_o, U_o = o.random_start(prng.random_block(5, p["n"], qe))
    want_tol = 1e-10 if prec == ae.PREC_FP64 else 1e-5
    for step in range(3):
        ctx.correct(1)
        th, U, pr = gpu_state(ctx)
        lam_o, U_o = o.correction(0, lam_o, U_o)
        err = np.abs(th / lam_o - 1)
        print("step %d: max relative difference %.2e (wanted %.2e)" % (step + 1, err.max(), err[:q].max()))
        assert err[:q].max() < want_tol and err.max() < (5e-9 if prec == ae.PREC_FP64 else 1e-5), (step, th, lam_o)
    lam, ok = ctx.solve(tol=1e-10, max_steps=300)
    th, U, pr = gpu_state(ctx)
    assert ok, pr
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
