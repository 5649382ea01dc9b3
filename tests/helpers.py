"""Shared test helpers: dense brute force, cluster-aware subspace comparison."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


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


def gap_prefixes(lam, q, gap=1e-2):
    """Prefix sizes m <= q after which the spectrum has a relative gap >= gap."""
    out = []
    for m in range(1, min(q, len(lam) - 1) + 1):
        if lam[m] / lam[m - 1] - 1.0 >= gap:
            out.append(m)
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


def compare_subspaces(lam_ref, Uref, U, M, q, gap=1e-2):
    """Max over gap-delimited prefixes m <= q of sin angle between the m-dim subspaces."""
    worst = 0.0
    for m in gap_prefixes(lam_ref, q, gap):
        worst = max(worst, sin_angle_M(Uref[:, :m], U[:, :m], M))
    return worst
