"""Pins of the oracle's eigensolver (Algorithms 3.1 / 3.2) against results the
mathematics fixes independently: dense brute force, a closed-form spectrum,
fixed points, Ritz bounds and multigrid contraction."""
import numpy as np
import pytest

from oracle import Oracle, guard_count
from workloads import configs
from tests.helpers import brute_force, compare_subspaces, mats

SMALL = [
    ("square16", lambda: configs.square(16, q=6)),
    ("lshape8j", lambda: configs.lshape(8, q=6, jitter_seed=5)),
    ("cube8", lambda: configs.cube(8, q=32)),  # the whole 32-member low cluster
    ("osc24", lambda: configs.oscillator(24, q=6)),  # closed shells 1+2+3
]


@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("smoother", ["gs", "mcgs", "l1jacobi", "chebyshev"])
def test_converges_to_dense_brute_force(name, make, smoother):
    p = make()
    A, M = mats(p)
    q = p["q"]
    full, _ = brute_force(p, min(p["n"], 3 * q + 10))
    qe = guard_count(full, q)
    o = Oracle(A, M, q=q, qe=qe, coarse_max=max(40, 3 * qe), smoother=smoother)
    lam, U, info = o.solve(tol=1e-11, max_steps=200)
    assert info["rho"][:q].max() <= 1e-11
    ref, Uref = brute_force(p, o.qe + 1)
    assert np.abs(lam[:q] / ref[:q] - 1).max() < 1e-10
    worst, ms = compare_subspaces(ref, Uref, U, M, q, qe=o.qe)
    assert worst < 1e-6, (worst, ms)
    assert np.abs(U.T @ (M @ U) - np.eye(o.qe)).max() < 1e-12


def test_lumped_mass_closed_form():
    """M = h^2 I on the Courant mesh: lambda_kl = 4/h^2 (sin^2(k pi h/2) + sin^2(l pi h/2))."""
    m = 32
    p = configs.square_lumped(m, q=8)
    A, M = mats(p)
    h = 1.0 / m
    k = np.arange(1, m)
    s = np.sin(k * np.pi * h / 2) ** 2
    exact = np.sort((4 / h ** 2) * (s[:, None] + s[None, :]).ravel())
    o = Oracle(A, M, q=8, coarse_max=100)
    lam, U, info = o.solve(tol=1e-11)
    assert np.abs(lam[:8] / exact[:8] - 1).max() < 1e-11


def test_random_start_matches_nested_start():
    p = configs.config(0)
    A, M = mats(p)
    o = Oracle(A, M, q=4, coarse_max=130, smoother="l1jacobi")
    U0 = configs.initial_block(p, o.qe)
    l1, U1, _ = o.solve(tol=1e-11, start="random", U0=U0)
    l2, U2, _ = o.solve(tol=1e-11, start="nested")
    assert np.abs(l1[:4] / l2[:4] - 1).max() < 1e-12
    ref = np.array([19.78679229, 49.55252612, 49.66736125, 79.71606372])
    assert np.abs(l1[:4] - ref).max() < 1e-7


def test_each_step_keeps_m_orthonormality_and_ritz_bounds():
    p = configs.lshape(8, q=5, jitter_seed=7)
    A, M = mats(p)
    o = Oracle(A, M, q=5, qe=6, coarse_max=30, smoother="l1jacobi")
    ref, _ = brute_force(p, 6)
    lam, U = o.random_start(configs.initial_block(p, 6, seed=11))
    prev = lam.copy()
    for _ in range(8):
        assert np.abs(U.T @ (M @ U) - np.eye(6)).max() < 1e-12
        assert np.all(lam >= ref * (1 - 1e-12))  # Poincare: Ritz values bound from above
        lam, U = o.correction(0, lam, U)
        assert np.all(lam <= prev * (1 + 1e-12))  # non-increasing
        prev = lam.copy()


def test_exact_eigenpairs_are_a_fixed_point():
    p = configs.square(12, q=4)
    A, M = mats(p)
    o = Oracle(A, M, q=4, qe=4, coarse_max=40)
    ref, Uref = brute_force(p, 5)
    lam, U = o.correction(0, ref[:4].copy(), Uref[:, :4].copy())
    assert np.abs(lam / ref[:4] - 1).max() < 1e-13
    assert compare_subspaces(ref, Uref, U, M, 4, qe=4)[0] < 1e-10


@pytest.mark.parametrize("smoother,bound", [("gs", 0.25), ("mcgs", 0.25), ("l1jacobi", 0.45), ("chebyshev", 0.15)])
def test_vcycle_is_symmetric_a_norm_contraction(smoother, bound):
    """The V-cycle as an affine iteration x -> x + B (b - A x): B symmetric and
    ||I - B A||_A < 1 (with textbook-sized factors for the 5-point Laplacian)."""
    p = configs.square(32)
    A, M = mats(p)
    o = Oracle(A, M, q=1, coarse_max=40, smoother=smoother)
    n = p["n"]
    rng = np.random.default_rng(0)

    def B(r):
        return o.vcycle(0, r, np.zeros_like(r))

    x = rng.standard_normal((n, 1))
    y = rng.standard_normal((n, 1))
    assert abs((x.T @ B(y)) - (y.T @ B(x))).max() < 1e-10 * abs(x.T @ B(x)).max()
    e = rng.standard_normal((n, 1))
    rate = 1.0
    for _ in range(25):
        e_new = e - B(A @ e)
        rate = np.sqrt((e_new.T @ (A @ e_new)) / (e.T @ (A @ e))).item()
        e = e_new / np.sqrt((e_new.T @ (A @ e_new)).item())
    assert rate < bound, rate


def test_gauss_seidel_rate_close_to_paper_example_1():
    """Example 1 with Gauss-Seidel V(1,1): the paper reports an average
    reduction of about 0.11 per correction (Table 1).  On a 127^2 grid with a
    ~500-point coarse space the oracle's rate is of that order."""
    p = configs.square(128, q=4)
    A, M = mats(p)
    o = Oracle(A, M, q=4, coarse_max=600, smoother="gs")
    lam, U, info = o.solve(tol=1e-11, record=True)
    r = [h[1][:4].max() for h in info["history"]]
    rate = (r[-1] / r[1]) ** (1.0 / (len(r) - 2))
    assert rate < 0.25, rate


def test_guard_rule():
    assert guard_count([1, 2, 3, 4, 5, 6], 3) == 3
    assert guard_count([1, 2, 3, 3.001, 3.002, 6, 7, 8], 3) == 5
    assert guard_count([1, 1, 1, 1, 1, 1, 1, 1, 1, 1], 2, cap=5) == 5


def test_relative_residual_closed_form():
    """u = e1 + eps e2 for M-orthonormal eigenvectors (lumped mass M = h^2 I):
    theta = (l1 + eps^2 l2)/(1 + eps^2) and
    rho = sqrt((l1 - theta)^2 + eps^2 (l2 - theta)^2) / (theta sqrt(1 + eps^2))."""
    m = 16
    p = configs.square_lumped(m, q=2)
    A, M = mats(p)
    l, E = brute_force(p, 2)
    o = Oracle(A, M, q=2, qe=2, coarse_max=40)
    for eps in (1e-3, 0.3):
        u = (E[:, 0] + eps * E[:, 1])[:, None]
        th = (l[0] + eps ** 2 * l[1]) / (1 + eps ** 2)
        want = np.sqrt((l[0] - th) ** 2 + eps ** 2 * (l[1] - th) ** 2) / (th * np.sqrt(1 + eps ** 2))
        got = o.residuals(0, np.array([th]), u)[0]
        assert abs(got / want - 1) < 1e-9


@pytest.mark.parametrize("degree,lo", [(1, 0.25), (2, 0.25), (3, 0.1)])
def test_chebyshev_smoother_is_the_scaled_chebyshev_polynomial(degree, lo):
    """With b = 0 the Chebyshev smoother maps the error e to p(D^-1 A) e, where
    p(t) = T_s((theta - t) / delta) / T_s(theta / delta) on [lo, 1] (theta, delta
    the interval's centre and half-width, T_s the Chebyshev polynomial of the
    first kind).  Checked against that closed form through the eigendecomposition
    of the symmetric D^-1/2 A D^-1/2, with T_s evaluated by cos / cosh."""
    p = configs.square(8)
    A, M = mats(p)
    o = Oracle(A, M, q=1, coarse_max=20, smoother="chebyshev", cheb_degree=degree, cheb_lo=lo)
    L = o.levels[0]
    n = p["n"]
    E = o._smooth(L, np.zeros((n, n)), np.eye(n), backward=False)
    Ad = L.A.toarray()
    d = np.asarray(L.l1, dtype=float).ravel()
    S = Ad / np.sqrt(d)[:, None] / np.sqrt(d)[None, :]
    lam, Q = np.linalg.eigh(S)
    assert lam.max() <= 1.0 + 1e-12 and lam.min() > 0  # the l1 scaling bounds the spectrum by 1

    def cheb_t(s, x):
        x = np.asarray(x, dtype=float)
        out = np.empty_like(x)
        inside = np.abs(x) <= 1
        out[inside] = np.cos(s * np.arccos(x[inside]))
        xo = x[~inside]
        out[~inside] = np.sign(xo) ** s * np.cosh(s * np.arccosh(np.abs(xo)))
        return out

    theta, delta = 0.5 * (1 + lo), 0.5 * (1 - lo)
    pl = cheb_t(degree, (theta - lam) / delta) / cheb_t(degree, np.array([theta / delta]))[0]
    E_ref = (Q * pl) @ Q.T
    E_ref = E_ref / np.sqrt(d)[:, None] * np.sqrt(d)[None, :]  # D^-1/2 p(S) D^1/2
    assert np.abs(E - E_ref).max() < 1e-12
    # the scaled polynomial is bounded by 1 / T_s(theta / delta) on [lo, 1]
    on = (lam >= lo)
    assert np.abs(pl[on]).max() <= 1.0 / cheb_t(degree, np.array([theta / delta]))[0] + 1e-14


def test_eig_pencil_range_restriction_on_dependent_basis():
    """Rayleigh-Ritz (Algorithm 3.1 step 2) on a basis with dependent columns:
    B = [B1, B1 C] makes the projected mass matrix M^ = B^T M B singular, and
    the oracle's small solver then restricts the pencil to the range of M^.
    With A, M positive definite the projected pencil's finite eigenpairs are
    those of (B1^T A B1, B1^T M B1) on the independent basis B1, so dense brute
    force there fixes both the values and the spanned subspace."""
    import scipy.linalg as sla
    from tests.helpers import sin_angle_M
    p = configs.square(12, q=4)
    A, M = mats(p)
    rng = np.random.default_rng(3)
    B1 = rng.standard_normal((p["n"], 9))
    B = np.hstack([B1, B1 @ rng.standard_normal((9, 3))])
    Ah = B.T @ (A @ B)
    Mh = B.T @ (M @ B)
    # precondition: M^ is singular to rounding, so the Cholesky branch is not taken
    try:
        c = np.linalg.cholesky(0.5 * (Mh + Mh.T))
        assert (np.diag(c) ** 2).min() <= 1e-13 * np.diag(Mh).max()
    except np.linalg.LinAlgError:
        pass
    mu, X = Oracle.eig_pencil(Ah, Mh, 5)
    ref, Y = sla.eigh(B1.T @ (A @ B1), B1.T @ (M @ B1), subset_by_index=[0, 5])
    assert np.abs(mu / ref[:5] - 1).max() < 1e-9
    V = B @ X
    assert np.abs(V.T @ (M @ V) - np.eye(5)).max() < 1e-9
    assert ref[5] / ref[4] - 1 > 1e-2  # the 5-dimensional subspace is isolated
    assert sin_angle_M(B1 @ Y[:, :5], V, M) < 1e-7


@pytest.mark.parametrize("shift", [0.0, 15.0])
def test_many_cycles_approach_the_exact_linear_solve(shift):
    """m AMG cycles of Algorithm 3.1 from the initial value U (eq. (3.2)) form a
    convergent iteration for the linear equation (3.1), so with m large the
    correction equals the Rayleigh-Ritz step on the exact solution
    (A - sigma M)^-1 (lambda - sigma) M U, formed here by a sparse direct solve;
    one cycle stays far from it."""
    import scipy.sparse.linalg as spla
    p = configs.square(24, q=4)
    A, M = mats(p)
    kw = dict(q=4, qe=4, coarse_max=60, smoother="gs", shift=shift)
    o1, o80 = Oracle(A, M, **kw), Oracle(A, M, cycles=80, **kw)
    lam, U = o1.nested_start()
    rhs = (M @ U) * (lam - shift)[None, :]
    V = spla.spsolve((A - shift * M).tocsc(), rhs)
    mu_exact, U_exact = o1.rayleigh_ritz(0, V)
    mu80, U80 = o80.correction(0, lam, U)
    mu1, _ = o1.correction(0, lam, U)
    assert np.abs(mu80 / mu_exact - 1).max() < 1e-11
    assert np.abs(mu1 / mu_exact - 1).max() > 1e3 * np.abs(mu80 / mu_exact - 1).max()
