"""Degenerate and boundary cases of the solve on the GPU, through the C ABI,
against dense brute force:
  - a positive semidefinite mass matrix (every seventh unknown carries no
    mass: the pencil has infinite eigenvalues there, the wanted finite ones are
    the largest eigenvalues mu of M x = mu A x inverted, lambda = 1 / mu);
  - the smallest problems the block width admits (a whole problem inside one
    workgroup's rows, a ragged last tile everywhere)."""
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import paper_1503_08462_amd as ae
from workloads import configs
from tests.helpers import brute_force, compare_subspaces, gap_prefixes, mats, sin_angle_M

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _solve(rowptr, col, a, m, q, tol, **kw):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = ae.Context(rowptr, col, a, m, q, ae.defaults(**kw))
    ctx.bind()
    lam, ok = ctx.solve(tol=tol, max_steps=300)
    pr = ctx.progress()
    qe = ctx.info()["qe"]
    U = ctx.iterate().cpu().numpy()[:, :qe].copy()
    ctx.close()
    return lam, ok, pr, U


@pytest.mark.parametrize("prec", [ae.PREC_FP64, ae.PREC_MIXED], ids=["fp64", "mixed"])
def test_semidefinite_mass_matches_brute_force(prec):
    p = configs.square(32, q=4)
    n, q = p["n"], 4
    keep = np.ones(n)
    keep[::7] = 0.0
    rows = np.repeat(np.arange(n), np.diff(p["rowptr"]))
    m2 = p["M"] * keep[rows] * keep[p["col"]]
    A, _ = mats(p)
    M2 = sp.csr_matrix((m2, p["col"], p["rowptr"]), shape=(n, n))
    # brute force on the definite pencil (M2, A): x^T A x = 1, M2 x = mu A x
    mu, X = sla.eigh(M2.toarray(), A.toarray())
    order = np.argsort(-mu)[: q + 4]
    lam_ref = 1.0 / mu[order]
    XA = X[:, order]  # A-orthonormal eigenvectors
    _say("semidefinite mass, N=%d, %d massless unknowns, prec=%d" % (n, int((keep == 0).sum()), prec))
    lam, ok, pr, U = _solve(p["rowptr"], p["col"], p["A"], m2, q, 1e-10, coarse_max=130, precision=prec)
    assert ok, pr
    tol = 1e-10 if prec == ae.PREC_FP64 else 1e-6
    assert np.abs(lam / lam_ref[:q] - 1).max() < tol, (lam, lam_ref[:q])
    # subspaces in the A inner product (M2 is only a seminorm)
    ms = gap_prefixes(lam_ref, q)
    assert ms, "no gap-delimited prefix to compare"
    for m in ms:
        assert sin_angle_M(XA[:, :m], U[:, :m], A) < 1e-6
    Uq = U[:, :q]
    assert np.abs(Uq.T @ (M2 @ Uq) - np.eye(q)).max() < 1e-10
    R = A @ Uq - (M2 @ Uq) * lam[None, :]
    assert (np.linalg.norm(R, axis=0) / (lam * np.linalg.norm(M2 @ Uq, axis=0))).max() <= 1e-10 * 1.01


@pytest.mark.parametrize("m,q,cm", [(9, 3, 20), (10, 2, 20), (12, 1, 30)])
def test_smallest_admissible_problems(m, q, cm):
    p = configs.square(m, q=q)
    _say("tiny square N=%d q=%d coarse_max=%d" % (p["n"], q, cm))
    lam_ref, Uref = brute_force(p, min(p["n"], q + 6))
    lam, ok, pr, U = _solve(p["rowptr"], p["col"], p["A"], p["M"], q, 1e-10, coarse_max=cm,
                            precision=ae.PREC_FP64)
    assert ok, pr
    assert np.abs(lam / lam_ref[:q] - 1).max() < 1e-10
    _, M = mats(p)
    worst, ms = compare_subspaces(lam_ref, Uref, U, M, q, qe=U.shape[1])
    print("compared prefixes", ms, "sin", worst)
    assert worst < 1e-6
