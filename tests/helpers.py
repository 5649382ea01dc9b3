"""Shared test helpers: dense brute force, an independent reference spectrum,
cluster-aware subspace comparison."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def mats(p):
    n = p["n"]
    A = sp.csr_matrix((p["A"], p["col"], p["rowptr"]), shape=(n, n))
    M = sp.csr_matrix((p["M"], p["col"], p["rowptr"]), shape=(n, n))
    A.sort_indices()
    M.sort_indices()
    return A, M


def brute_force(p, count):
    A, M = mats(p)
    return sla.eigh(A.toarray(), M.toarray(), subset_by_index=[0, count - 1])


def reference_eigenvalues(p, count):
    """The `count` smallest eigenvalues of (A, M), ascending: dense LAPACK for
    N <= 2500, else shift-invert Lanczos about 0 (ARPACK through SciPy).  Both
    are library solvers independent of the oracle and of the HIP path; used to
    place the cluster gaps that decide which subspaces are comparable."""
    A, M = mats(p)
    if p["n"] <= 2500:
        return sla.eigh(A.toarray(), M.toarray(), eigvals_only=True, subset_by_index=[0, count - 1])
    lam = spla.eigsh(A.tocsc(), k=count, M=M.tocsc(), sigma=0.0, which="LM", return_eigenvectors=False,
                     ncv=max(2 * count + 1, count + 20))
    return np.sort(lam)


def gap_prefixes(lam, q, qe=None, gap=1e-2):
    """Prefix sizes m after which the reference spectrum lam has a relative gap
    lam[m] / lam[m-1] - 1 >= gap: every such m <= q, and, when the q-th value
    lies inside a cluster that the block of qe columns holds entirely, the end
    of that cluster (the first such m in (q, qe])."""
    ok = lambda m: len(lam) > m and lam[m] / lam[m - 1] - 1.0 >= gap
    out = [m for m in range(1, min(q, len(lam) - 1) + 1) if ok(m)]
    if qe is not None and not ok(q):
        for m in range(q + 1, qe + 1):
            if ok(m):
                out.append(m)
                break
    return out


def sin_angle_M(Uref, U, M):
    """Largest sine of the principal angles between span(U) and span(Uref) in the
    M inner product (Uref M-orthonormal); ||(I - Uref Uref^T M) U||_M for U
    M-orthonormalised."""
    U = np.asarray(U, dtype=np.float64)
    G = U.T @ (M @ U)
    L = np.linalg.cholesky(0.5 * (G + G.T))
    Un = np.linalg.solve(L, U.T).T
    W = Un - Uref @ (Uref.T @ (M @ Un))
    S = W.T @ (M @ W)
    return float(np.sqrt(max(0.0, np.linalg.eigvalsh(0.5 * (S + S.T)).max())))


def compare_subspaces(lam_ref, Uref, U, M, q, qe=None, gap=1e-2, min_prefixes=1):
    """Largest sine of the angle between the m-dimensional leading subspaces of
    Uref and U over the gap-delimited prefixes of lam_ref (gap_prefixes), and
    the list of prefix sizes compared.  Fails when fewer than `min_prefixes`
    prefixes qualify, so that a check never passes by comparing nothing."""
    ms = gap_prefixes(lam_ref, q, qe, gap)
    assert len(ms) >= min_prefixes, "no gap-delimited prefix to compare (q=%d, qe=%s)" % (q, qe)
    worst = 0.0
    for m in ms:
        worst = max(worst, sin_angle_M(Uref[:, :m], U[:, :m], M))
    return worst, ms
