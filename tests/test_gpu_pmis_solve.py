"""Solves on a hierarchy set up on the device (coarsening = PMIS: strength,
PMIS splitting with the parallel second pass, direct interpolation, transpose and Galerkin products formed on
the GPU level by level).  The hierarchy changes, the eigenpairs of (A, M) do
not: the converged eigenvalues match dense LAPACK (or shift-invert Lanczos)
and the eigenvectors span the same subspaces; the library's first splitting
equals the oracle's PMIS with the same SplitMix64 random parts."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1503_08462_amd as ae
from oracle.amg import pmis_splitting
from workloads import configs
from workloads.prng import uniform01
from tests.helpers import brute_force, compare_subspaces, mats, reference_eigenvalues

pytestmark = pytest.mark.gpu

SEED = 7


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("lshape24j", lambda: configs.lshape(24, q=10, jitter_seed=2), 300, True),
    ("cube12", lambda: configs.cube(12, q=8), 100, True),
    ("oscillator40", lambda: configs.oscillator(40, q=10), 150, True),
    ("oscillator200", lambda: configs.oscillator(200, q=10), 300, False),
]


@pytest.mark.parametrize("name,make,cm,dense", CASES, ids=[c[0] for c in CASES])
def test_solve_on_device_hierarchy(name, make, cm, dense):
    import torch
    p = make()
    q, n = p["q"], p["n"]
    opts = ae.defaults(coarse_max=cm, coarsening=ae.COARSEN_PMIS, coarsen_seed=SEED)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], q, opts)
    info = ctx.info()
    _say("pmis solve %s: levels %s, qe %d" % (name, info["dims"].tolist(), info["qe"]))
    # the first level's splitting is the oracle's PMIS on the same random parts
    rp, ci, a, _ = ctx.level_matrix(0)
    A0 = sp.csr_matrix((a, ci, rp), shape=(n, n))
    cf_o, _, _ = pmis_splitting(A0, uniform01(SEED, np.arange(n)), opts.theta, second_pass=True)
    assert np.array_equal(ctx.splitting(0), cf_o)
    ctx.bind()
    U = torch.zeros((n, q), dtype=torch.float64, device="cuda")
    lam, ok = ctx.solve(tol=1e-10, max_steps=300, U_out=U)
    torch.cuda.synchronize()
    assert ok
    pr = ctx.progress()
    _say("pmis solve %s: %d corrections" % (name, pr["steps"]))
    A, M = mats(p)
    if dense:
        qe = ctx.info()["qe"]
        ref, Uref = brute_force(p, qe + 1)
        assert np.abs(lam / ref[:q] - 1).max() < 1e-10
        Ufull = ctx.iterate().cpu().numpy()[:, :qe]
        worst, ms = compare_subspaces(ref, Uref, Ufull, M, q, qe=qe)
        _say("compared prefixes %s, largest sine %.2e" % (ms, worst))
        assert worst < 1e-6
    else:
        ref = reference_eigenvalues(p, q)
        assert np.abs(lam / ref - 1).max() < 1e-9
    Ug = U.cpu().numpy()
    assert np.abs(Ug.T @ (M @ Ug) - np.eye(q)).max() < 1e-12
    ctx.close()


@pytest.mark.parametrize("variant", ["mixed", "gauss_seidel"])
def test_solve_on_device_hierarchy_variants(variant):
    """The device-built hierarchy under the other forms of the correction: the
    FP32 V-cycle under the FP64 residual, and the multicolour Gauss-Seidel
    smoother (its colouring is taken on the device-built levels)."""
    import torch
    p = configs.lshape(40, q=8, jitter_seed=3)
    q, n = p["q"], p["n"]
    kw = dict(coarse_max=300, coarsening=ae.COARSEN_PMIS, coarsen_seed=SEED + 1)
    if variant == "mixed":
        kw["precision"] = ae.PREC_MIXED
    else:
        kw["smoother"] = ae.SMOOTH_GAUSS_SEIDEL
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], q, ae.defaults(**kw))
    ctx.bind()
    U = torch.zeros((n, q), dtype=torch.float64, device="cuda")
    lam, ok = ctx.solve(tol=1e-9, max_steps=300, U_out=U)
    torch.cuda.synchronize()
    assert ok
    _say("pmis %s: levels %s, %d corrections" % (variant, ctx.info()["dims"].tolist(), ctx.progress()["steps"]))
    ref = reference_eigenvalues(p, q)
    assert np.abs(lam / ref - 1).max() < 1e-9
    _, M = mats(p)
    Ug = U.cpu().numpy()
    assert np.abs(Ug.T @ (M @ Ug) - np.eye(q)).max() < 1e-12
    ctx.close()
