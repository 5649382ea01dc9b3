"""Dense symmetric-definite eigen-decomposition on the device (the coarsest
eigen-solve of the hierarchy) through the C ABI, against LAPACK (SciPy's eigh)
on seeded pencils and on a coarsest level of the host setup: eigenvalues,
Z^T M Z = I and Z^T A Z = Lambda; a mass matrix that is not positive definite
is refused."""
import sys
import time

import numpy as np
import pytest
import scipy.linalg as sla

import paper_1503_08462_amd as ae
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _check(torch, A, M, label):
    n = A.shape[0]
    t0 = time.perf_counter()
    lam, Z, sweeps = ae.dense_sygv(torch.from_numpy(A).cuda(), torch.from_numpy(M).cuda())
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    lam, Z = lam.cpu().numpy(), Z.cpu().numpy()
    ref = sla.eigh(A, M, eigvals_only=True)
    scale = np.abs(ref).max()
    err = np.abs(lam - ref).max() / scale
    orth = np.abs(Z.T @ M @ Z - np.eye(n)).max()
    diag = np.abs(Z.T @ A @ Z - np.diag(lam)).max() / scale
    _say("%s: n %d, %d sweeps, %.1f ms, eigenvalues %.1e, Z^T M Z %.1e, Z^T A Z %.1e" %
         (label, n, sweeps, ms, err, orth, diag))
    assert np.all(np.diff(lam) >= 0)
    assert err < 1e-12 and orth < 1e-11 and diag < 1e-12
    return lam


@pytest.mark.parametrize("n", [1, 2, 7, 64, 257, 512])
def test_dense_sygv_random_pencils(n):
    import torch
    rng = np.random.default_rng(100 + n)
    X = rng.standard_normal((n, n))
    A = X @ X.T + 0.1 * np.eye(n)
    Y = rng.standard_normal((n, n))
    M = Y @ Y.T / n + np.eye(n)
    _check(torch, np.ascontiguousarray(A), np.ascontiguousarray(M), "random")


def test_dense_sygv_coarsest_level_of_host_setup():
    import torch
    p = configs.oscillator(200, q=10)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=700, qe=12))
    nl = ctx.info()["levels"]
    rp, ci, a, m = ctx.level_matrix(nl - 1)
    host_lam = ctx.coarse_eigenvalues()
    ctx.close()
    n = rp.size - 1
    A = np.zeros((n, n))
    M = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, ci] = a
    M[rows, ci] = m
    A = 0.5 * (A + A.T)
    M = 0.5 * (M + M.T)
    lam = _check(torch, A, M, "coarsest oscillator200")
    assert np.abs(lam - host_lam).max() <= 1e-12 * np.abs(host_lam).max()


def test_dense_sygv_refuses_indefinite_mass():
    import torch
    n = 5
    A = np.eye(n)
    M = np.eye(n)
    M[3, 3] = -1.0
    with pytest.raises(ae.AmgEigError) as e:
        ae.dense_sygv(torch.from_numpy(A).cuda(), torch.from_numpy(M).cuda())
    assert e.value.code == ae.ENOTSPD
