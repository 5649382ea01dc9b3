"""Pins of the oracle's AMG setup (Section 2) against hand derivations and
structural facts that the paper's level sizes fix."""
import numpy as np
import scipy.sparse as sp

from oracle import amg
from workloads import configs
from tests.helpers import mats


def _lap1d(n):
    return sp.csr_matrix(2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))


def test_1d_laplacian_hand_derived_hierarchy():
    """RS first pass on tridiag(-1,2,-1), N = 7, picks every other point; direct
    interpolation gives weights 1/2 and the Galerkin operator is tridiag(-1/2,1,-1/2)."""
    A = _lap1d(7)
    cf, S = amg.rs_splitting(A, 0.25)
    assert cf.tolist() == [0, 1, 0, 1, 0, 1, 0]
    P = amg.direct_interpolation(A, S, cf).toarray()
    want = np.array([[.5, 0, 0], [1, 0, 0], [.5, .5, 0], [0, 1, 0], [0, .5, .5], [0, 0, 1], [0, 0, .5]])
    assert np.array_equal(P, want)
    A2 = amg.galerkin(sp.csr_matrix(P), A).toarray()
    assert np.allclose(A2, np.array([[1, -.5, 0], [-.5, 1, -.5], [0, -.5, 1]]), atol=0, rtol=0)
    M2 = amg.galerkin(sp.csr_matrix(P), sp.identity(7, format="csr")).toarray()
    assert np.allclose(M2, np.array([[1.5, .25, 0], [.25, 1.5, .25], [0, .25, 1.5]]), atol=0, rtol=0)


def test_strength_threshold_eq_2_1():
    # row 0: couplings -4 (strong), -1 (= 0.25 * 4, strong by >=), -0.5 (weak), +3 (never)
    A = sp.csr_matrix(np.array([[10., -4, -1, -.5, 3], [-4, 10, 0, 0, 0], [-1, 0, 10, 0, 0],
                                [-.5, 0, 0, 10, 0], [3, 0, 0, 0, 10]]))
    S = amg.strength(A, 0.25).toarray()
    assert S[0].tolist() == [0, 1, 1, 0, 0]
    assert S[4].tolist() == [0, 0, 0, 0, 0]  # only a positive coupling: S_i empty


def test_level2_is_half_of_five_point_grids():
    """The paper's level-2 sizes are (N+1)/2 (red-black split) on its 5-point grids."""
    for p in (configs.square(64), configs.lshape(16), configs.quadrants(16)):
        A, _ = mats(p)
        cf, _ = amg.rs_splitting(A, 0.25)
        assert cf.sum() == (p["n"] + 1) // 2, p["meta"]


def test_f_points_have_strong_c_neighbour_and_constants_interpolate():
    for p in (configs.lshape(12, jitter_seed=4), configs.cube(8), configs.oscillator(20)):
        A, M = mats(p)
        cf, S = amg.rs_splitting(A, 0.25)
        P = amg.direct_interpolation(A, S, cf)
        Sd = S.tolil().rows
        for i in np.flatnonzero(cf == 0):
            if Sd[i]:
                assert cf[Sd[i]].max() == 1, i
        # rows with zero row sum (away from the Dirichlet boundary) interpolate 1 exactly
        rowsum = np.asarray(A.sum(axis=1)).ravel()
        scale = np.abs(A).sum(axis=1).A.ravel()
        zero = np.abs(rowsum) < 1e-12 * scale
        p1 = P @ np.ones(P.shape[1])
        if p["meta"]["family"] != "oscillator":
            assert zero.sum() > 0
        assert np.abs(p1[zero] - 1).max(initial=0) < 1e-13
        # Galerkin operators stay symmetric
        A2 = amg.galerkin(P, A)
        M2 = amg.galerkin(P, M)
        assert abs(A2 - A2.T).max() < 1e-12 * abs(A2).max()
        assert abs(M2 - M2.T).max() < 1e-12 * abs(M2).max()


def test_hierarchy_galerkin_chain_identity():
    from oracle import Oracle
    p = configs.lshape(10, jitter_seed=1)
    A, M = mats(p)
    o = Oracle(A, M, q=4, coarse_max=30)
    assert len(o.levels) >= 3
    dn = o.levels[-1].n
    Q = o.prolong_from_coarsest(0, np.eye(dn))
    assert np.abs(Q.T @ (M @ Q) - o.levels[-1].M.toarray()).max() < 1e-14
    assert np.abs(Q.T @ (A @ Q) - o.levels[-1].A.toarray()).max() < 1e-12
    R = o.restrict_to_coarsest(0, M @ Q)
    assert np.abs(R - Q.T @ (M @ Q)).max() < 1e-14


def test_rs_first_pass_measure_updates_on_asymmetric_strength():
    """Hand-traced first pass where the decrement of the measure matters.

    Strong dependencies (i -> j means j in S_i): 1,2,3 -> 0; 0 -> 4; 5 -> 4;
    4 -> 5; 9 -> 5; 7,8 -> 6.  Measures |S^T|: 0:3, 4:2, 5:2, 6:2.
    0 becomes C, 1,2,3 F; 0 depends on the undecided 4, whose measure drops to 1.
    Then 5 (measure 2, lowest index) becomes C and 4, 9 become F; finally 6 is C.
    Without the decrement 4 would win the tie and the result would be C = {0,4,6,9}.
    """
    edges = {1: [0], 2: [0], 3: [0], 0: [4], 5: [4], 4: [5], 9: [5], 7: [6], 8: [6]}
    A = 10 * np.eye(10)
    for i, js in edges.items():
        for j in js:
            A[i, j] = -1.0
    cf, _ = amg.rs_splitting(sp.csr_matrix(A), 0.25, second_pass=False)
    assert np.flatnonzero(cf).tolist() == [0, 5, 6]


def _strong(n, deps):
    rows = [i for i, js in deps.items() for _ in js]
    cols = [j for i, js in deps.items() for j in js]
    S = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    S.sort_indices()
    return S


def test_rs_second_pass_hand_traced():
    """F point 1 depends on C point 0 and on F point 2, which depends only on
    1 and C point 3: no common strong C point, so 2 becomes C.  In the second
    case F point 1 has two such F neighbours (2 and 4): 1 itself becomes C."""
    from oracle import native
    S = _strong(5, {1: [0, 2], 2: [1, 3]})
    cf = native.rs_second_pass(S, np.array([1, 0, 0, 1, 0]))
    assert cf.tolist() == [1, 0, 1, 1, 0]
    S = _strong(6, {1: [0, 2, 4], 2: [1, 3], 4: [1, 5]})
    cf = native.rs_second_pass(S, np.array([1, 0, 0, 1, 0, 1]))
    assert cf.tolist() == [1, 1, 0, 1, 0, 1]


def test_second_pass_gives_common_c_points():
    """After coarsening, every strongly coupled F-F pair shares a strong C point."""
    for p in (configs.lshape(20, jitter_seed=2), configs.cube(8)):
        A, _ = mats(p)
        cf, S = amg.rs_splitting(A, 0.25)
        Sl = S.tolil().rows
        for i in np.flatnonzero(cf == 0):
            Ci = {k for k in Sl[i] if cf[k] == 1}
            for j in Sl[i]:
                if cf[j] == 0:
                    assert Ci & set(Sl[j]), (i, j)


def test_pmis_1d_laplacian_picks_every_other_point():
    """PMIS on tridiag(-1,2,-1), N = 7: interior points weigh 2 + r_i, the ends
    1 + r_i.  With equal random parts (ties to the larger index), increasing or
    decreasing ones, the rounds traced by hand take C = {1, 3, 5} in three
    rounds, the textbook coarsening of the 1D Laplacian."""
    A = _lap1d(7)
    for r in (np.full(7, 0.5), np.arange(7) / 10.0, (6 - np.arange(7)) / 10.0):
        cf, S, rounds = amg.pmis_splitting(A, r, 0.25)
        assert cf.tolist() == [0, 1, 0, 1, 0, 1, 0]
        assert rounds == 3


def test_pmis_marks_f_along_dependence_not_influence():
    """Asymmetric strength, traced by hand: S_0 = {1}, S_1 = {0, 2}, S_2 = {3},
    S_3 = {2} (point 1 depends on 2, 2 does not depend on 1).  Point 2 (weight
    2 + r_2) becomes C first; 1 and 3 depend on it and become F; 0 is then a
    lone undecided point and becomes C: [1, 0, 1, 0] in two rounds.  Marking F
    along the other direction (points that 2 depends on) would leave 1
    undecided and make it C."""
    A = sp.csr_matrix(np.array([[2.0, -1, 0, 0], [-1, 2, -0.3, 0], [0, -0.3, 11, -10], [0, 0, -10, 11]]))
    cf, S, rounds = amg.pmis_splitting(A, np.array([0.1, 0.5, 0.0, 0.0]), 0.25)
    assert [list(S.indices[S.indptr[i]:S.indptr[i + 1]]) for i in range(4)] == [[1], [0, 2], [3], [2]]
    assert cf.tolist() == [1, 0, 1, 0] and rounds == 2


def test_pmis_invariants_on_workloads():
    """On seeded random parts: every point decided; every F point that some
    point depends on depends strongly on a C point; the first round's C set,
    the local maxima of the weights over the symmetrised strength graph
    (formed here with sparse products), is contained in C."""
    from workloads.prng import uniform01
    for p in (configs.cube(10, q=4), configs.lshape(16, q=4, jitter_seed=1), configs.quadrants(12, q=4)):
        A, _ = mats(p)
        n = A.shape[0]
        r = uniform01(77, np.arange(n))
        cf, S, rounds = amg.pmis_splitting(A, r, 0.25)
        assert set(np.unique(cf).tolist()) <= {0, 1} and rounds >= 1
        nst = np.asarray(S.sum(axis=0)).ravel()
        dep_c = np.asarray(S @ cf.astype(float)).ravel()
        assert np.all(dep_c[(cf == 0) & (nst > 0)] > 0)
        assert np.all(cf[nst == 0] == 0)
        w = nst + r
        G = ((S + S.T) != 0).tocoo()
        beats = (w[G.col] > w[G.row]) | ((w[G.col] == w[G.row]) & (G.col > G.row))
        beaten = np.zeros(n, bool)
        beaten[G.row[beats & (nst[G.col] > 0)]] = True
        first = (nst > 0) & ~beaten
        assert first.any() and np.all(cf[first] == 1)


def test_pmis_second_pass_promotes_the_heavier_of_a_conflict():
    """Path 0-1-2-3 with cf = [C, F, F, C]: F points 1 and 2 depend on each
    other and share no strong C point (S_1 cap C = {0}, S_2 cap C = {3}), so the
    heavier of the two becomes C; afterwards no conflict is left."""
    A = _lap1d(4)
    S = amg.strength(A, 0.25)
    cf = np.array([1, 0, 0, 1])
    out, rounds = amg.pmis_second_pass(S, cf, np.array([1.0, 2.1, 2.7, 1.0]))
    assert out.tolist() == [1, 0, 1, 1] and rounds == 1
    out, rounds = amg.pmis_second_pass(S, cf, np.array([1.0, 2.9, 2.7, 1.0]))
    assert out.tolist() == [1, 1, 0, 1] and rounds == 1
    out, rounds = amg.pmis_second_pass(S, np.array([0, 1, 0, 1]), np.ones(4))
    assert out.tolist() == [0, 1, 0, 1] and rounds == 0


def test_pmis_second_pass_leaves_no_conflict():
    """After the second pass every F point j in S_i of an F point i shares a
    strong C point with it (checked with sparse products: (S_C S_C^T)_ij > 0
    for S_C = S restricted to C columns), and the first pass's C points stay C."""
    from workloads.prng import uniform01
    for p in (configs.cube(10, q=4), configs.lshape(16, q=4, jitter_seed=1), configs.oscillator(30, q=4)):
        A, _ = mats(p)
        n = A.shape[0]
        r = uniform01(3, np.arange(n))
        cf1, S, _ = amg.pmis_splitting(A, r, 0.25)
        cf2, _, _ = amg.pmis_splitting(A, r, 0.25, second_pass=True)
        assert np.all(cf2[cf1 == 1] == 1) and cf2.sum() >= cf1.sum()
        SC = S @ sp.diags((cf2 == 1).astype(float))
        common = (SC @ SC.T).toarray()
        Ff = S.tocoo()
        sel = (cf2[Ff.row] == 0) & (cf2[Ff.col] == 0) & (Ff.row != Ff.col)
        assert np.all(common[Ff.row[sel], Ff.col[sel]] > 0)
