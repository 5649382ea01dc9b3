"""Oracle AMG setup (Section 2 of the paper), plain FP64 on the CPU.

Test infrastructure only: the eigensolver library never imports this.

  strength            eq. (2.1): S_i = {j != i : -a_ij >= theta * max_{l != i, a_il < 0} |a_il|}
  rs_splitting        Section 2.1: classical Ruge-Stueben coarsening (first pass
                      on |S_i^T|, then the second pass giving strongly
                      coupled F points a common strong C point)
  pmis_splitting      a parallel C/F splitting (PMIS: parallel modified
                      independent set, De Sterck, Yang and Heys 2006) on the
                      same strength graph, the parallel coarsening that
                      replaces the sequential Ruge-Stueben passes on a GPU,
                      optionally followed by a parallel form of the RS
                      second pass (pmis_second_pass)
  direct_interpolation eq. (2.2)-(2.4) with P_i = S_i intersect C
  galerkin            eq. (2.5): A_{k+1} = P^T A_k P, M_{k+1} = P^T M_k P
  build_hierarchy     the level loop of Section 2.3
  coarse_eigen        the small generalized eigenproblem on the coarsest level
  colouring           first-fit colouring of a level's matrix graph and the
                      colour-ordered row sequence of the multicolour
                      Gauss-Seidel smoother (a reordering of the paper's
                      Gauss-Seidel smoothing, Section 4.1)
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import native


def csr(rowptr, col, val, n):
    m = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col, np.int64), np.asarray(rowptr, np.int64)),
                      shape=(n, n))
    m.sort_indices()
    return m


def _rows(A):
    return np.repeat(np.arange(A.shape[0], dtype=np.int64), np.diff(A.indptr))


def strength(A, theta=0.25):
    """Strong-dependence matrix S (pattern only, CSR), eq. (2.1).

    Only negative off-diagonal couplings can be strong; a row without negative
    off-diagonals has S_i empty.
    """
    n = A.shape[0]
    rows = _rows(A)
    cols = A.indices.astype(np.int64)
    neg = (cols != rows) & (A.data < 0)
    mx = np.zeros(n)
    np.maximum.at(mx, rows[neg], -A.data[neg])
    strong = neg & (-A.data >= theta * mx[rows])
    S = sp.csr_matrix((np.ones(int(strong.sum())), (rows[strong], cols[strong])), shape=(n, n))
    S.sort_indices()
    return S


def rs_splitting(A, theta=0.25, second_pass=True):
    """C/F splitting (1 = C, 0 = F) by classical Ruge-Stueben coarsening."""
    S = strength(A, theta)
    ST = S.T.tocsr()
    ST.sort_indices()
    cf = native.rs_first_pass(S, ST)
    if second_pass:
        cf = native.rs_second_pass(S, cf)
    return cf, S


def pmis_second_pass(S, cf, w):
    """Parallel form of the Ruge-Stueben second pass on a splitting cf.

    A conflict is a pair of F points (i, j) with j in S_i that share no C point
    strongly influencing both (S_i cap S_j cap C empty).  Each round, for every
    conflict the heavier point of the pair, by (w, index), becomes C; rounds
    repeat until no conflict is left.  Returns (cf, rounds).
    """
    n = S.shape[0]
    cf = np.array(cf, dtype=np.int64)
    rounds = 0
    while True:
        promote = set()
        for i in range(n):
            if cf[i] != 0:
                continue
            Si = S.indices[S.indptr[i]:S.indptr[i + 1]]
            Ci = set(int(k) for k in Si if cf[k] == 1)
            for j in Si:
                if cf[j] != 0 or j == i:
                    continue
                Sj = S.indices[S.indptr[j]:S.indptr[j + 1]]
                if not any(int(k) in Ci for k in Sj):
                    promote.add(i if (w[i], i) > (w[j], j) else int(j))
        if not promote:
            return cf, rounds
        rounds += 1
        for k in promote:
            cf[k] = 1


def pmis_splitting(A, r, theta=0.25, second_pass=False):
    """C/F splitting (1 = C, 0 = F) by PMIS on the strength graph of eq. (2.1).

    r holds one random number in [0, 1) per point, drawn by the caller.  Point
    i weighs w_i = |S_i^T| + r_i, the number of points that depend strongly on
    it plus its random part; points that no point depends on start as F, the
    others undecided.  Each round, every undecided point whose (w_i, i) exceeds
    (w_j, j) for all undecided neighbours j in the symmetrised strength graph
    (j in S_i or i in S_j) becomes C, then every undecided point that depends
    strongly on one of the new C points becomes F.  Rounds repeat until no
    point is undecided; each round makes at least the heaviest undecided point
    C.  With second_pass, pmis_second_pass follows on the same weights (its
    rounds are not counted).  Returns (cf, S, rounds).
    """
    n = A.shape[0]
    S = strength(A, theta)
    ST = S.T.tocsr()
    ST.sort_indices()
    G = ((S + ST) != 0).tocsr()
    G.sort_indices()
    w = np.diff(ST.indptr).astype(np.float64) + np.asarray(r, dtype=np.float64)
    state = np.where(np.diff(ST.indptr) == 0, 0, -1)
    rounds = 0
    while (state == -1).any():
        rounds += 1
        undecided = [i for i in range(n) if state[i] == -1]
        new_c = []
        for i in undecided:
            nbrs = [j for j in G.indices[G.indptr[i]:G.indptr[i + 1]] if j != i and state[j] == -1]
            if all((w[j], j) < (w[i], i) for j in nbrs):
                new_c.append(i)
        new_set = set(new_c)
        for i in new_c:
            state[i] = 1
        for i in undecided:
            if state[i] == -1 and any(j in new_set for j in S.indices[S.indptr[i]:S.indptr[i + 1]]):
                state[i] = 0
    cf = state.astype(np.int64)
    if second_pass:
        cf, _ = pmis_second_pass(S, cf, w)
    return cf, S, rounds


def direct_interpolation(A, S, cf):
    """Prolongation P (N x n_C) by direct interpolation, eq. (2.2)-(2.4).

    C points are injected.  An F point i interpolates from P_i = S_i cap C with
        w_ij = -alpha_i a_ij / a~_ii,
        alpha_i = (sum_{j in N_i, a_ij < 0} a_ij) / (sum_{l in P_i} a_il).
    S_i holds negative couplings only, so the positive-coupling term of (2.3)
    has no interpolation points; positive off-diagonals are added to the
    diagonal instead, a~_ii = a_ii + sum_{j in N_i, a_ij > 0} a_ij, which keeps
    constants exact for zero row-sum rows.  F points with P_i empty get an
    empty row.
    """
    n = A.shape[0]
    cidx = np.cumsum(cf) - 1
    rows = _rows(A)
    cols = A.indices.astype(np.int64)
    v = A.data
    off = cols != rows
    diag = np.zeros(n)
    np.add.at(diag, rows[~off], v[~off])
    sum_neg = np.zeros(n)
    np.add.at(sum_neg, rows[off & (v < 0)], v[off & (v < 0)])
    sum_pos = np.zeros(n)
    np.add.at(sum_pos, rows[off & (v > 0)], v[off & (v > 0)])
    # entries of S restricted to C columns, from F rows
    Sr = _rows(S)
    Sc = S.indices.astype(np.int64)
    # look up a_ij for each strong (i, j)
    Akey = rows * n + cols
    Skey = Sr * n + Sc
    pos = np.searchsorted(Akey, Skey)
    a_s = v[pos]
    sel = (cf[Sr] == 0) & (cf[Sc] == 1)
    sum_P = np.zeros(n)
    np.add.at(sum_P, Sr[sel], a_s[sel])
    alpha = np.divide(sum_neg, sum_P, out=np.zeros(n), where=sum_P != 0)
    ahat = diag + sum_pos
    w = -alpha[Sr[sel]] * a_s[sel] / ahat[Sr[sel]]
    c_rows = np.flatnonzero(cf == 1)
    pr = np.concatenate([c_rows, Sr[sel]])
    pc = np.concatenate([cidx[c_rows], cidx[Sc[sel]]])
    pv = np.concatenate([np.ones(c_rows.size), w])
    P = sp.csr_matrix((pv, (pr, pc)), shape=(n, int(cf.sum())))
    P.sort_indices()
    return P


def galerkin(P, A):
    """P^T A P, eq. (2.5)."""
    C = (P.T @ A @ P).tocsr()
    C.sort_indices()
    return C


class Level:
    def __init__(self, A, M):
        self.A, self.M = A, M
        self.P = None
        self.cf = None
        self.n = A.shape[0]


def build_hierarchy(A, M, theta=0.25, coarse_max=512, coarse_min=8, max_levels=25, stall=0.9):
    """Levels 1..n (index 0 = finest).  Coarsening stops once d_k <= coarse_max,
    when the next level would be smaller than coarse_min, or when it would keep
    more than ``stall`` of the points."""
    levels = [Level(A, M)]
    while len(levels) < max_levels and levels[-1].n > coarse_max:
        L = levels[-1]
        cf, S = rs_splitting(L.A, theta)
        nc = int(cf.sum())
        if nc < coarse_min or nc > stall * L.n or nc == 0:
            break
        P = direct_interpolation(L.A, S, cf)
        L.P, L.cf = P, cf
        levels.append(Level(galerkin(P, L.A), galerkin(P, L.M)))
    return levels


def coarse_eigen(levels):
    """All eigenpairs of (A_n, M_n): Z^T M_n Z = I, Z^T A_n Z = diag(lam)."""
    An = levels[-1].A.toarray()
    Mn = levels[-1].M.toarray()
    lam, Z = sla.eigh(0.5 * (An + An.T), 0.5 * (Mn + Mn.T))
    return lam, Z


def colouring(A):
    """Colours of a level for multicolour Gauss-Seidel: i and j are neighbours
    when a_ij != 0 or a_ji != 0 (i != j); rows 0..n-1 in turn take the smallest
    colour no coloured neighbour holds.  Returns (colour, order) where order
    lists the rows colour by colour, ascending within a colour, so that a
    Gauss-Seidel sweep in that order updates each colour's rows from values of
    other colours only."""
    S = sp.csr_matrix(A, copy=True)
    S.setdiag(0.0)
    S.eliminate_zeros()
    S.data[:] = 1.0
    G = (S + S.T).tocsr()
    G.sort_indices()
    colour, _ = native.greedy_colour(G)
    order = np.argsort(colour, kind="stable").astype(np.int64)
    return colour, order
