"""Pins of the oracle's shifted correction equation (Remark 3.1): the linear
equation of Algorithm 3.1 as (A_k - sigma M_k) u~ = (lambda - sigma) M_k u.
Checked against what fixes it independently: a direct sparse solve of the
shifted system, the fixed points of the correction (the exact eigenpairs),
dense brute force for the converged pairs, and the unshifted oracle at
sigma = 0."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import Oracle
from workloads import configs
from tests.helpers import brute_force, compare_subspaces, mats


def test_zero_shift_is_the_unshifted_solver():
    p = configs.lshape(12, q=4, jitter_seed=1)
    A, M = mats(p)
    a = Oracle(A, M, q=4, qe=6, coarse_max=60, smoother="chebyshev").solve(tol=1e-10)
    b = Oracle(A, M, q=4, qe=6, coarse_max=60, smoother="chebyshev", shift=0.0).solve(tol=1e-10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("smoother", ["gs", "mcgs", "chebyshev"])
def test_shifted_vcycle_solves_the_shifted_system(smoother):
    """Iterating x <- x + B (b - (A - sigma M) x) with B the shifted V-cycle
    reaches the direct solution of (A - sigma M) x = b; B is symmetric."""
    p = configs.lshape(16, q=2, jitter_seed=4)
    A, M = mats(p)
    o0 = Oracle(A, M, q=2, qe=2, coarse_max=60)
    sigma = 0.8 * o0.lam_n[0]
    o = Oracle(A, M, q=2, qe=2, coarse_max=60, smoother=smoother, shift=sigma)
    K = (A - sigma * M).tocsc()
    rng = np.random.default_rng(3)
    b = rng.standard_normal((p["n"], 2))
    exact = spla.splu(K).solve(b)
    x = np.zeros_like(b)
    for _ in range(60):
        x = x + o.vcycle(0, b - K @ x, np.zeros_like(b))
    assert np.abs(x - exact).max() < 1e-9 * np.abs(exact).max()
    u, v = rng.standard_normal((p["n"], 1)), rng.standard_normal((p["n"], 1))
    Bu, Bv = o.vcycle(0, u, np.zeros_like(u)), o.vcycle(0, v, np.zeros_like(v))
    assert abs((v.T @ Bu - u.T @ Bv).item()) < 1e-10 * abs((u.T @ Bu).item())


def test_exact_eigenpairs_are_a_fixed_point_of_the_shifted_correction():
    p = configs.square(12, q=4)
    A, M = mats(p)
    ref, Uref = brute_force(p, 5)
    o = Oracle(A, M, q=4, qe=4, coarse_max=40, shift=0.5 * ref[0])
    lam, U = o.correction(0, ref[:4].copy(), Uref[:, :4].copy())
    assert np.abs(lam / ref[:4] - 1).max() < 1e-13
    assert compare_subspaces(ref, Uref, U, M, 4, qe=4)[0] < 1e-10


@pytest.mark.parametrize("smoother", ["gs", "chebyshev"])
def test_shifted_solve_converges_to_brute_force(smoother):
    p = configs.lshape(16, q=6, jitter_seed=2)
    A, M = mats(p)
    ref, Uref = brute_force(p, 12)
    o0 = Oracle(A, M, q=6, qe=8, coarse_max=80, smoother=smoother)
    o = Oracle(A, M, q=6, qe=8, coarse_max=80, smoother=smoother, shift=0.5 * o0.lam_n[0])
    lam, U, info = o.solve(tol=1e-11, max_steps=200)
    assert info["rho"][:6].max() <= 1e-11
    assert np.abs(lam[:6] / ref[:6] - 1).max() < 1e-10
    assert compare_subspaces(ref, Uref, U, M, 6, qe=8)[0] < 1e-6


def test_shift_saves_corrections():
    """With a shift the error of u_j shrinks by about (lambda_j - sigma) /
    (lambda_{qe+1} - sigma) per exact solve instead of lambda_j / lambda_{qe+1};
    on the oscillator (q = 10 wanted of a 16-wide block) sigma = 0.9 lambda_1
    of the coarsest level saves a fifth of the corrections (52 -> 42)."""
    p = configs.oscillator(48, q=10)
    A, M = mats(p)
    base = Oracle(A, M, q=10, qe=16, coarse_max=150, smoother="gs")
    steps0 = base.solve(tol=1e-10, max_steps=300)[2]["steps"]
    o = Oracle(A, M, q=10, qe=16, coarse_max=150, smoother="gs", shift=0.9 * base.lam_n[0])
    lam, U, info = o.solve(tol=1e-10, max_steps=300)
    ref, _ = brute_force(p, 11)
    assert np.abs(lam[:10] / ref[:10] - 1).max() < 1e-10
    assert info["steps"] <= 0.85 * steps0, (info["steps"], steps0)


def test_shift_above_the_coarsest_eigenvalue_is_rejected():
    p = configs.square(12, q=2)
    A, M = mats(p)
    lam1 = Oracle(A, M, q=2, qe=2, coarse_max=40).lam_n[0]
    with pytest.raises(np.linalg.LinAlgError):
        Oracle(A, M, q=2, qe=2, coarse_max=40, shift=1.01 * lam1)
