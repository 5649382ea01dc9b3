"""Named synthetic workloads (seeded; shapes and structure of the paper's examples).

Each builder returns a dict with the CSR pattern shared by A and M
(``rowptr`` int64, ``col`` int32), ``A`` and ``M`` (float64), ``n``, the number
of wanted eigenpairs ``q`` and a ``meta`` dict describing the recipe.

  square(m)          -Lap on (0,1)^2, h = 1/m, (m-1)^2 unknowns (paper Ex. 1 family)
  square_lumped(m)   same stiffness with the row-sum (lumped) mass M = h^2 I
  lshape(m, jitter)  -Lap on the L-shape, h = 1/m, (2m-1)^2 - m^2 unknowns (Ex. 2 family)
  cube(m)            -div(kappa grad) on (0,1)^3, Kuhn tets, 4x4x4 checkerboard
                     kappa in {1, 1e3}, (m-1)^3 unknowns
  oscillator(m)      -Lap + (x^2+y^2) on (-6,6)^2, (m-1)^2 unknowns
  quadrants(m, ...)  -div(K grad) on (-1,1)^2 with per-quadrant K (Ex. 3 / Ex. 4)
"""
import numpy as np

from . import fem, prng


def _pack(rowptr, col, a, m, q, meta):
    return {"rowptr": rowptr, "col": col, "A": a, "M": m, "n": rowptr.size - 1, "q": q, "meta": meta}


def square(m, q=4):
    xy, tris, bnd, used, _ = fem.unit_square(m)
    rowptr, col, a, mm, _ = fem.assemble_2d(xy, tris, bnd)
    return _pack(rowptr, col, a, mm, q, {"family": "square", "m": m, "h": 1.0 / m})


def square_lumped(m, q=4):
    p = square(m, q)
    rowptr, col = p["rowptr"], p["col"]
    rows = np.repeat(np.arange(p["n"]), np.diff(rowptr))
    lumped = np.where(rows == col, (1.0 / m) ** 2, 0.0)
    p["M"] = lumped
    p["meta"] = dict(p["meta"], family="square_lumped")
    return p


def lshape(m, q=10, jitter_seed=None, amp=0.2):
    xy, tris, bnd, used, _ = fem.lshape(m)
    if jitter_seed is not None:
        xy = fem.jitter_nodes(xy, ~bnd, 1.0 / m, jitter_seed, amp)
    rowptr, col, a, mm, _ = fem.assemble_2d(xy, tris, bnd)
    return _pack(rowptr, col, a, mm, q, {"family": "lshape", "m": m, "h": 1.0 / m,
                                         "jitter_seed": jitter_seed, "amp": amp})


def cube(m, q=20, kappa_hi=1e3):
    xyz, tets, bnd, tcell = fem.unit_cube_kuhn(m)
    centre = (tcell + 0.5) / m
    blk = np.floor(4.0 * centre).astype(np.int64).sum(axis=1)
    kappa = np.where(blk % 2 == 0, 1.0, kappa_hi)
    rowptr, col, a, mm, _ = fem.assemble_3d(xyz, tets, bnd, kappa)
    return _pack(rowptr, col, a, mm, q, {"family": "cube", "m": m, "h": 1.0 / m, "kappa_hi": kappa_hi})


def oscillator(m, q=64, half_width=6.0):
    xy, tris, bnd, used, _ = fem.box(m, -half_width, half_width)
    rowptr, col, a, mm, _ = fem.assemble_2d(xy, tris, bnd, potential=True)
    return _pack(rowptr, col, a, mm, q, {"family": "oscillator", "m": m, "h": 2 * half_width / m})


def quadrants(m, q=13, k_ur=1e3, k_ll=1e-3, k_off=1.0):
    """(-1,1)^2, h = 1/m; K = k_ur on [0,1]^2, k_ll on [-1,0]^2, k_off elsewhere."""
    xy, tris, bnd, used, tcell = fem.box(2 * m, -1.0, 1.0)
    cx = (tcell[:, 0] + 0.5) / m - 1.0
    cy = (tcell[:, 1] + 0.5) / m - 1.0
    kappa = np.full(tris.shape[0], k_off)
    kappa[(cx > 0) & (cy > 0)] = k_ur
    kappa[(cx < 0) & (cy < 0)] = k_ll
    rowptr, col, a, mm, _ = fem.assemble_2d(xy, tris, bnd, kappa)
    return _pack(rowptr, col, a, mm, q, {"family": "quadrants", "m": m, "h": 1.0 / m})


# ------------------------------------------------------------- the five workloads
def config(idx, scale=1.0):
    """The five workloads at full size (scale=1) or shrunk in mesh parameter.

    0: unit square, 31x31 interior (N = 961), q = 4, random start seed 1
    1: jittered L-shape, h = 1/256 (N = 195 585), q = 10, jitter/start seed 2
    2: 3D checkerboard cube, 100^3 cells (N = 970 299), q = 20, seed 3
    3: oscillator on (-6,6)^2, 2048^2 cells (N = 4 190 209), q = 64, seed 4
    """
    if idx == 0:
        p = square(max(4, int(round(32 * scale))), q=4); p["seed"] = 1
    elif idx == 1:
        p = lshape(max(4, int(round(256 * scale))), q=10, jitter_seed=2); p["seed"] = 2
    elif idx == 2:
        p = cube(max(8, 4 * int(round(25 * scale))), q=20); p["seed"] = 3
    elif idx == 3:
        p = oscillator(max(16, int(round(2048 * scale))), q=64); p["seed"] = 4
    else:
        raise ValueError(idx)
    return p


def initial_block(p, qe, seed=None):
    """Seeded U(-1,1) start block, N x qe row-major."""
    return prng.random_block(p.get("seed", 1) if seed is None else seed, p["n"], qe)


# ------------------------------------------------------------ serving stream (C5)
def lshape_m_for(n_target):
    # N = (2m-1)^2 - m^2 = 3m^2 - 4m + 1
    return max(4, int(round((4 + np.sqrt(16 - 12 * (1 - n_target))) / 6)))


def guard_width(family, q):
    """Block width a client asks for so that the block never ends inside a
    cluster of the family's spectrum (extra pairs computed beside the wanted
    ones): the oscillator's eigenvalues 2(k+1) have multiplicity k+1, so the
    width is the end of the cluster holding the q-th; the checkerboard cube has
    a low cluster of 32 (one mode per kappa = 1 block), so widths below 32 take
    the whole cluster; the L-shape has no multiple eigenvalues, and a quarter
    more pairs keep the convergence factor lambda_q / lambda_{qe+1} small."""
    if family == "oscillator":
        k, total = 0, 0
        while total < q:
            k += 1
            total += k
        return total
    if family == "cube":
        return 32 if q < 32 else q + 4
    return q + max(2, (q + 3) // 4)


def request_stream(n_requests=256, seed=5, n_lo=10_000, n_hi=1_000_000):
    """Seeded request descriptors: family, mesh parameter, q, block width qe,
    per-request seed."""
    out = []
    for r in range(n_requests):
        rs = prng.derive_seed(seed, r)
        u = prng.uniform01(rs, np.arange(4, dtype=np.uint64))
        fam = ("lshape", "cube", "oscillator")[min(2, int(u[0] * 3))]
        nt = n_lo + u[1] * (n_hi - n_lo)
        q = (4, 8, 16, 32)[min(3, int(u[2] * 4))]
        if fam == "lshape":
            m = lshape_m_for(nt)
        elif fam == "cube":
            m = max(8, int(round(nt ** (1.0 / 3.0))) + 1)
            m = 4 * max(2, int(round(m / 4)))  # checkerboard blocks stay whole cells
        else:
            m = max(16, int(round(np.sqrt(nt))) + 1)
        out.append({"id": r, "family": fam, "m": m, "q": q, "qe": guard_width(fam, q), "seed": rs,
                    "u_arrival": float(u[3])})
    return out


def build_request(req):
    fam, m, q = req["family"], req["m"], req["q"]
    if fam == "lshape":
        p = lshape(m, q=q, jitter_seed=req["seed"] & 0xFFFFFFFF)
    elif fam == "cube":
        p = cube(m, q=q)
    else:
        p = oscillator(m, q=q)
    p["seed"] = req["seed"]
    p["qe"] = req["qe"]
    return p
