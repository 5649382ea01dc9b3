"""Oracle AMG multilevel-correction eigensolver (Section 3), plain FP64 CPU.

Test infrastructure only: the eigensolver library never imports this, and it
never touches a GPU.  It follows the paper's formulation directly:

  vcycle        the AMG iteration of (3.2): one V-cycle, nu_pre / nu_post
                smoothing sweeps, exact solve on the coarsest level
  correction    Algorithm 3.1: block inexact inverse iteration (3.1)-(3.2),
                then Rayleigh-Ritz on V_n + span{V} with the block matrices
                A_{n,k}, M_{n,k} and the eigenproblem (3.3)
  solve         Algorithm 3.2: eigen-solve on the coarsest level, prolongate,
                one correction per level, then corrections on the finest level
                until the relative residual criterion holds

Shift (Remark 3.1): with shift = sigma the linear equation of Algorithm 3.1
becomes (A_k - sigma M_k) u~ = (lambda - sigma) M_k u, solved by the AMG
iteration of the shifted operators A_k - sigma M_k on the same hierarchy (the
coarsest solve with A_n - sigma M_n).  sigma must lie below the smallest
eigenvalue for these operators to stay positive definite.

Smoothers: "gs" (the paper's Gauss-Seidel: forward before, backward after the
coarse correction), "mcgs" (the same sweeps with the rows of each level taken
colour by colour, amg.colouring), "l1jacobi" (x += D^-1 (b - A x), d_i = sum_j |a_ij|) and
"chebyshev" (degree-s Chebyshev polynomial in D^-1 A for the l1 diagonal D,
on the interval [lo, 1]; 1 bounds the spectrum of D^-1 A by Gershgorin since
d_i = a_ii + sum_{j != i} |a_ij|).
"""
import numpy as np
import scipy.linalg as sla

from . import amg, native


def guard_count(lam, q, gap=1e-2, cap=None):
    """Smallest m >= q with lam[m] / lam[m-1] - 1 >= gap (1-based m), capped.

    Implements the paper's 'compute extra eigenpairs' strategy (Section 4.5)
    as a rule on approximate eigenvalues: a wanted set must not end inside a
    cluster."""
    lam = np.asarray(lam)
    cap = (2 * q + 8) if cap is None else cap
    cap = min(cap, lam.size - 1)
    m = q
    while m < cap and lam[m] / lam[m - 1] - 1.0 < gap:
        m += 1
    return m


class Oracle:
    def __init__(self, A, M, q, qe=None, theta=0.25, coarse_max=512, coarse_min=None, max_levels=25,
                 smoother="gs", nu_pre=1, nu_post=1, cheb_degree=2, cheb_lo=0.25,
                 guard_gap=1e-2, shift=0.0, cycles=1):
        self.q = q
        self.cycles = int(cycles)  # m of Algorithm 3.1: AMG cycles per correction
        cmin = coarse_min if coarse_min is not None else 2 * (qe if qe else q) + 2
        self.levels = amg.build_hierarchy(A, M, theta, coarse_max, cmin, max_levels)
        self.lam_n, self.Z = amg.coarse_eigen(self.levels)
        self.qe = qe if qe is not None else guard_count(self.lam_n, q, guard_gap)
        self.smoother = smoother
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.cheb_degree = cheb_degree
        self.cheb_lo = cheb_lo
        self.shift = float(shift)
        for L in self.levels:  # the operator of the linear equation on each level
            L.As = (L.A - self.shift * L.M).tocsr() if self.shift != 0.0 else L.A
        An = self.levels[-1].As.toarray()
        self._coarse_chol = sla.cho_factor(0.5 * (An + An.T))  # fails unless A_n - sigma M_n is SPD
        for L in self.levels:
            d = np.zeros(L.n)
            np.add.at(d, amg._rows(L.As), np.abs(L.As.data))
            L.l1 = d
            L.diag = L.As.diagonal()
            if smoother == "mcgs":
                L.colour, L.order = amg.colouring(L.As)
        self.history = []

    # ------------------------------------------------------------------ smoothing
    def _smooth(self, L, b, x, backward):
        if self.smoother == "gs":
            x = np.ascontiguousarray(x, dtype=np.float64).copy()
            return native.gs_sweep(L.As, b, x, backward=backward)
        if self.smoother == "mcgs":
            x = np.ascontiguousarray(x, dtype=np.float64).copy()
            return native.gs_sweep(L.As, b, x, backward=backward, order=L.order)
        if self.smoother == "l1jacobi":
            return x + (b - L.As @ x) / L.l1[:, None]
        if self.smoother == "chebyshev":
            theta = 0.5 * (1.0 + self.cheb_lo)
            delta = 0.5 * (1.0 - self.cheb_lo)
            # Chebyshev acceleration (Saad, Iterative Methods, 2nd ed., Alg. 12.1) on D^-1 A
            sigma = theta / delta
            rho_k = 1.0 / sigma
            r = (b - L.As @ x) / L.l1[:, None]
            d = r / theta
            for _ in range(self.cheb_degree):
                x = x + d
                r = r - (L.As @ d) / L.l1[:, None]
                rho_n = 1.0 / (2.0 * sigma - rho_k)
                d = rho_n * rho_k * d + (2.0 * rho_n / delta) * r
                rho_k = rho_n
            return x
        raise ValueError(self.smoother)

    def vcycle(self, k, b, x):
        """One V-cycle for A_k x = b (A_k - sigma M_k with a shift) from initial
        guess x (the AMG iteration of (3.2))."""
        L = self.levels[k]
        for _ in range(self.nu_pre):
            x = self._smooth(L, b, x, backward=False)
        r = b - L.As @ x
        rc = L.P.T @ r
        if k + 1 == len(self.levels) - 1:
            ec = sla.cho_solve(self._coarse_chol, rc)
        else:
            ec = self.vcycle(k + 1, rc, np.zeros_like(rc))
        x = x + L.P @ ec
        for _ in range(self.nu_post):
            x = self._smooth(L, b, x, backward=True)
        return x

    # -------------------------------------------------------------- transfers
    def restrict_to_coarsest(self, k, W):
        """I_k^n W: apply P^T level by level from k down to the coarsest level."""
        for l in range(k, len(self.levels) - 1):
            W = self.levels[l].P.T @ W
        return W

    def prolong_from_coarsest(self, k, Y):
        """I_n^k Y: apply P level by level from the coarsest level up to k."""
        for l in range(len(self.levels) - 2, k - 1, -1):
            Y = self.levels[l].P @ Y
        return Y

    # ------------------------------------------------------------ Rayleigh-Ritz
    @staticmethod
    def eig_pencil(Ah, Mh, count):
        """Smallest ``count`` eigenpairs of Ah x = mu Mh x with x^T Mh x = 1.

        If Mh is numerically singular (V nearly inside the coarse space), the
        pencil is restricted to the range of Mh first."""
        Ah = 0.5 * (Ah + Ah.T)
        Mh = 0.5 * (Mh + Mh.T)
        try:
            c = np.linalg.cholesky(Mh)
            d = np.diag(c) ** 2
            if d.min() > 1e-13 * np.diag(Mh).max():
                mu, X = sla.eigh(Ah, Mh, subset_by_index=[0, count - 1])
                return mu, X
        except np.linalg.LinAlgError:
            pass
        s, Q = np.linalg.eigh(Mh)
        keep = s > 1e-13 * s.max()
        T = Q[:, keep] / np.sqrt(s[keep])
        mu, Y = np.linalg.eigh(T.T @ Ah @ T)
        return mu[:count], T @ Y[:, :count]

    def rayleigh_ritz(self, k, V):
        """Step 2 of Algorithm 3.1 for the block V on level k."""
        L = self.levels[k]
        dn = self.levels[-1].n
        AV = L.A @ V
        MV = L.M @ V
        BA = self.restrict_to_coarsest(k, AV)
        BM = self.restrict_to_coarsest(k, MV)
        Ah = np.block([[self.levels[-1].A.toarray(), BA], [BA.T, V.T @ AV]])
        Mh = np.block([[self.levels[-1].M.toarray(), BM], [BM.T, V.T @ MV]])
        mu, X = self.eig_pencil(Ah, Mh, self.qe)
        U = self.prolong_from_coarsest(k, X[:dn]) + V @ X[dn:]
        return mu, U

    def correction(self, k, lam, U):
        """Algorithm 3.1: AMGCorrection(n, k, {lam, U}), m = self.cycles AMG
        cycles on the linear equation (3.1) from the initial value U, eq. (3.2);
        with a shift sigma the right-hand side is (lam - sigma) M_k u (Remark 3.1)."""
        L = self.levels[k]
        rhs = (L.M @ U) * (lam - self.shift)[None, :]
        V = U
        for _ in range(self.cycles):
            V = self.vcycle(k, rhs, V)
        return self.rayleigh_ritz(k, V)

    # -------------------------------------------------------------- residuals
    def residuals(self, k, lam, U):
        """rho_j = ||A u_j - lam_j M u_j||_2 / (lam_j ||M u_j||_2)."""
        L = self.levels[k]
        MU = L.M @ U
        R = L.A @ U - MU * lam[None, :]
        return np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(MU, axis=0))

    # ----------------------------------------------------------------- driver
    def nested_start(self):
        """Algorithm 3.2 up to the finest level: coarsest eigenpairs, then one
        correction on each level n-1, ..., 2, and prolongation to level 1."""
        lam = self.lam_n[: self.qe].copy()
        U = self.Z[:, : self.qe].copy()
        for k in range(len(self.levels) - 2, 0, -1):
            U = self.levels[k].P @ U
            lam, U = self.correction(k, lam, U)
        U = self.levels[0].P @ U if len(self.levels) > 1 else U
        return lam, U

    def random_start(self, U0):
        """Rayleigh-Ritz of a seeded random block on V_n + span{U0}."""
        return self.rayleigh_ritz(0, np.asarray(U0, dtype=np.float64))

    def solve(self, tol=1e-8, max_steps=60, start="nested", U0=None, record=False):
        if len(self.levels) == 1:
            lam, U = self.lam_n[: self.qe], self.Z[:, : self.qe]
            return lam, U, {"steps": 0, "rho": self.residuals(0, lam, U)}
        lam, U = self.nested_start() if start == "nested" else self.random_start(U0)
        steps = 0
        hist = []
        while True:
            rho = self.residuals(0, lam, U)
            if record:
                hist.append((lam.copy(), rho.copy()))
            if rho[: self.q].max() <= tol or steps >= max_steps:
                break
            lam, U = self.correction(0, lam, U)
            steps += 1
        return lam, U, {"steps": steps, "rho": rho, "history": hist}
