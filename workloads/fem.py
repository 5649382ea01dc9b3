"""Seeded P1 finite-element test problems A u = lambda M u (inputs only).

Meshes are structured: 2D squares cut by the (1,-1) diagonal, i.e. the edge
from (x+h, y) to (x, y+h), and 3D cubes cut into the six Kuhn tetrahedra around
the (0,0,0)-(1,1,1) diagonal.  Dirichlet conditions are imposed by keeping only
interior nodes as unknowns.  A is the stiffness matrix of -div(kappa grad u)
(plus an optional potential mass term), M the consistent mass matrix; both are
returned on one shared CSR pattern (explicit zeros kept), sorted columns.

Element integrals are exact: for barycentric coordinates on a d-simplex T,
    int_T prod_i lambda_i^{a_i} = d! |T| prod_i a_i! / (sum_i a_i + d)!.
This module builds the eigenproblem's input; it holds none of the eigensolver.
"""
import math
import numpy as np

from . import prng


# --------------------------------------------------------------------------- CSR
def coo_to_csr(n, rows, cols, vals_list):
    """Sum duplicate (row, col) entries; one pattern for every value array."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * np.int64(n) + cols
    order = np.argsort(key, kind="stable")
    ks = key[order]
    first = np.empty(ks.shape[0], dtype=bool)
    first[:1] = True
    first[1:] = ks[1:] != ks[:-1]
    starts = np.flatnonzero(first)
    uk = ks[starts]
    r = uk // n
    c = uk - r * n
    out = [np.add.reduceat(np.asarray(v, dtype=np.float64)[order], starts) for v in vals_list]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(np.bincount(r, minlength=n))
    return rowptr, c.astype(np.int32), out


# ---------------------------------------------------------------------- 2D meshes
def rect_grid(nx, ny, x0, y0, h, cell_mask=None):
    """Nodes and (1,-1)-diagonal triangles of an nx-by-ny cell grid.

    Returns coordinates (n_nodes x 2), triangles (n_tri x 3, node indices),
    the boundary flag per node and the cell index (i, j) of each triangle.
    ``cell_mask[j, i]`` False removes cell (i, j).  A node is on the boundary if
    it lies on the outer rectangle or touches a removed cell.
    """
    if cell_mask is None:
        cell_mask = np.ones((ny, nx), dtype=bool)
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    node_id = jj * (nx + 1) + ii
    xy = np.stack([x0 + ii.ravel() * h, y0 + jj.ravel() * h], axis=1).astype(np.float64)
    cj, ci = np.nonzero(cell_mask)
    a = node_id[cj, ci]
    b = node_id[cj, ci + 1]
    c = node_id[cj + 1, ci]
    d = node_id[cj + 1, ci + 1]
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([b, d, c], 1)], 0)
    tcell = np.concatenate([np.stack([ci, cj], 1)] * 2, 0)
    used = np.zeros((ny + 1) * (nx + 1), dtype=bool)
    used[tris.ravel()] = True
    # a node is interior iff all four surrounding cells exist
    pad = np.zeros((ny + 2, nx + 2), dtype=bool)
    pad[1:-1, 1:-1] = cell_mask
    full = pad[:-1, :-1] & pad[:-1, 1:] & pad[1:, :-1] & pad[1:, 1:]
    boundary = ~full.ravel()
    boundary |= ~used
    return xy, tris, boundary, used, tcell


def unit_square(m):
    """Unit square (0,1)^2 with m cells per side, h = 1/m."""
    return rect_grid(m, m, 0.0, 0.0, 1.0 / m)


def lshape(m):
    """(-1,1)^2 minus [0,1) x (-1,0], h = 1/m (2m cells per side)."""
    ny = nx = 2 * m
    mask = np.ones((ny, nx), dtype=bool)
    mask[:m, m:] = False  # cells with x in [0,1), y in [-1,0)
    return rect_grid(nx, ny, -1.0, -1.0, 1.0 / m, mask)


def box(m, lo, hi):
    """Square (lo,hi)^2 with m cells per side."""
    return rect_grid(m, m, lo, lo, (hi - lo) / m)


def jitter_nodes(xy, movable, h, seed, amp=0.2):
    """Shift each movable node's coordinates by independent U(-amp h, amp h)."""
    xy = xy.copy()
    idx = np.flatnonzero(movable).astype(np.uint64)
    dx = prng.uniform_pm1(seed, 2 * idx) * (amp * h)
    dy = prng.uniform_pm1(seed, 2 * idx + np.uint64(1)) * (amp * h)
    xy[idx.astype(np.int64), 0] += dx
    xy[idx.astype(np.int64), 1] += dy
    return xy


def _simplex_moment(exps, dim):
    """int_T prod lambda^exps / |T| for a dim-simplex."""
    s = sum(exps)
    return math.factorial(dim) * np.prod([math.factorial(e) for e in exps]) / math.factorial(s + dim)


def _quartic_tensor_2d():
    """I4[i,j,k,l] = int_T lambda_i lambda_j lambda_k lambda_l / |T|."""
    t = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    e = [0, 0, 0]
                    for v in (i, j, k, l):
                        e[v] += 1
                    t[i, j, k, l] = _simplex_moment(e, 2)
    return t


def assemble_2d(xy, tris, boundary, kappa=None, potential=False):
    """P1 stiffness (+ optional (x^2+y^2) mass term) and consistent mass.

    kappa: per-triangle coefficient array or None (1).  Returns
    (rowptr, col, A, M, dof_nodes) with unknowns = non-boundary nodes in
    increasing node order.
    """
    n_nodes = xy.shape[0]
    dof = -np.ones(n_nodes, dtype=np.int64)
    dof_nodes = np.flatnonzero(~boundary)
    dof[dof_nodes] = np.arange(dof_nodes.size)
    n = dof_nodes.size
    p = xy[tris]  # T x 3 x 2
    e1 = p[:, 1] - p[:, 0]
    e2 = p[:, 2] - p[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * np.abs(det)
    g = np.empty((tris.shape[0], 3, 2))
    g[:, 1, 0] = e2[:, 1] / det
    g[:, 1, 1] = -e2[:, 0] / det
    g[:, 2, 0] = -e1[:, 1] / det
    g[:, 2, 1] = e1[:, 0] / det
    g[:, 0] = -g[:, 1] - g[:, 2]
    kap = np.ones(tris.shape[0]) if kappa is None else np.asarray(kappa, dtype=np.float64)
    K = (kap * area)[:, None, None] * np.einsum("tid,tjd->tij", g, g)
    Mloc = (area / 12.0)[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None]
    if potential:
        I4 = _quartic_tensor_2d()
        xx = np.einsum("tk,tl->tkl", p[:, :, 0], p[:, :, 0]) + np.einsum("tk,tl->tkl", p[:, :, 1], p[:, :, 1])
        K = K + area[:, None, None] * np.einsum("ijkl,tkl->tij", I4, xx)
    return _scatter(n, dof, tris, K, Mloc) + (dof_nodes,)


def _scatter(n, dof, cells, K, Mloc):
    nv = cells.shape[1]
    r = np.repeat(dof[cells], nv, axis=1).reshape(-1)
    c = np.tile(dof[cells], (1, nv)).reshape(-1)
    keep = (r >= 0) & (c >= 0)
    rowptr, col, (a, m) = coo_to_csr(n, r[keep], c[keep], [K.reshape(-1)[keep], Mloc.reshape(-1)[keep]])
    return rowptr, col, a, m


# ---------------------------------------------------------------------- 3D meshes
_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def unit_cube_kuhn(m):
    """Unit cube, m cells per side, each cube cut into 6 Kuhn tetrahedra."""
    h = 1.0 / m
    s = m + 1
    kk, jj, ii = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    xyz = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], 1)
    boundary = ((ii == 0) | (ii == m) | (jj == 0) | (jj == m) | (kk == 0) | (kk == m)).ravel()
    ck, cj, ci = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets, tcell = [], []
    for perm in _KUHN_PERMS:
        off = np.zeros((4, 3), dtype=np.int64)
        for step, axis in enumerate(perm):
            off[step + 1] = off[step]
            off[step + 1, axis] += 1
        verts = [((ck + o[2]) * s + (cj + o[1])) * s + (ci + o[0]) for o in off]
        tets.append(np.stack(verts, 1))
        tcell.append(np.stack([ci, cj, ck], 1))
    return xyz, np.concatenate(tets, 0), boundary, np.concatenate(tcell, 0)


def assemble_3d(xyz, tets, boundary, kappa=None, chunk=2_000_000):
    n_nodes = xyz.shape[0]
    dof = -np.ones(n_nodes, dtype=np.int64)
    dof_nodes = np.flatnonzero(~boundary)
    dof[dof_nodes] = np.arange(dof_nodes.size)
    n = dof_nodes.size
    rows, cols, kv, mv = [], [], [], []
    for s0 in range(0, tets.shape[0], chunk):
        t = tets[s0:s0 + chunk]
        p = xyz[t]
        J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns
        det = np.linalg.det(J)
        vol = np.abs(det) / 6.0
        Jinv = np.linalg.inv(J)  # rows are grad lambda_1..3
        g = np.empty((t.shape[0], 4, 3))
        g[:, 1:] = Jinv
        g[:, 0] = -Jinv.sum(axis=1)
        kap = np.ones(t.shape[0]) if kappa is None else np.asarray(kappa[s0:s0 + chunk], dtype=np.float64)
        K = (kap * vol)[:, None, None] * np.einsum("tid,tjd->tij", g, g)
        Ml = (vol / 20.0)[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None]
        r = np.repeat(dof[t], 4, axis=1).reshape(-1)
        c = np.tile(dof[t], (1, 4)).reshape(-1)
        keep = (r >= 0) & (c >= 0)
        rows.append(r[keep]); cols.append(c[keep])
        kv.append(K.reshape(-1)[keep]); mv.append(Ml.reshape(-1)[keep])
    rowptr, col, (a, m) = coo_to_csr(n, np.concatenate(rows), np.concatenate(cols),
                                     [np.concatenate(kv), np.concatenate(mv)])
    return rowptr, col, a, m, dof_nodes
