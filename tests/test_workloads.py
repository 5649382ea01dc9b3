"""Input-generator invariants (meshes, P1 assembly, counter-based PRNG)."""
import os

import numpy as np
import scipy.sparse as sp

from workloads import configs, fem, prng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mat(p, key):
    return sp.csr_matrix((p[key], p["col"], p["rowptr"]), shape=(p["n"], p["n"]))


def test_splitmix64_published_vector():
    want = [int(x) for x in open(os.path.join(GOLD, "splitmix64_seed1234567.txt")) if not x.startswith("#")]
    got = prng.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    assert [int(v) for v in got] == want


def test_random_block_layout_and_range():
    b = prng.random_block(7, 100, 3)
    assert b.shape == (100, 3) and b.min() >= -1 and b.max() < 1
    # column j does not depend on the block width
    assert np.array_equal(prng.random_block(7, 100, 5)[:, :3], b)


def test_sizes_of_the_five_workloads_at_small_scale():
    assert configs.config(0)["n"] == 961
    assert configs.lshape(8)["n"] == 15 ** 2 - 8 ** 2
    assert configs.cube(8)["n"] == 7 ** 3
    assert configs.oscillator(16)["n"] == 15 ** 2


def test_courant_mesh_stiffness_is_five_point_stencil():
    p = configs.square(8)
    A = _mat(p, "A").toarray()
    n1 = 7
    T = 2 * np.eye(n1) - np.eye(n1, k=1) - np.eye(n1, k=-1)
    L5 = np.kron(np.eye(n1), T) + np.kron(T, np.eye(n1))
    assert np.abs(A - L5).max() < 1e-14


def test_symmetry_and_mass_row_sums():
    for p in (configs.square(8), configs.lshape(6, jitter_seed=3), configs.cube(8), configs.oscillator(12)):
        A, M = _mat(p, "A"), _mat(p, "M")
        assert abs(A - A.T).max() < 1e-12 * abs(A).max()
        assert abs(M - M.T).max() < 1e-15
    # interior rows of the uniform square: consistent-mass row sum = h^2
    p = configs.square(8)
    rs = np.asarray(_mat(p, "M").sum(axis=1)).ravel()
    grid = rs.reshape(7, 7)
    assert np.allclose(grid[1:-1, 1:-1], (1 / 8) ** 2, rtol=1e-14)


def test_neumann_stiffness_annihilates_constants_and_potential_integral():
    # all nodes free (no boundary): A 1 = 0 for the Laplacian part, and the
    # potential mass integrates x^2 + y^2 exactly: sum_ij W_ij = int V = 3456
    xy, tris, bnd, used, _ = fem.box(12, -6.0, 6.0)
    free = np.zeros_like(bnd)
    rp, col, a, m, _ = fem.assemble_2d(xy, tris, free)
    A = sp.csr_matrix((a, col, rp))
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12
    rp, col, w, m, _ = fem.assemble_2d(xy, tris, free, potential=True)
    W = sp.csr_matrix((w - a, col, rp))
    assert abs(W.sum() - 2 * 12 * (2 * 6 ** 3 / 3)) < 1e-9
    assert abs(sp.csr_matrix((m, col, rp)).sum() - 144.0) < 1e-10
    # 3D: Kuhn mesh, constants in the kernel and total mass = volume
    xyz, tets, bnd3, _ = fem.unit_cube_kuhn(4)
    rp, col, a, m, _ = fem.assemble_3d(xyz, tets, np.zeros_like(bnd3))
    A = sp.csr_matrix((a, col, rp))
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12
    assert abs(m.sum() - 1.0) < 1e-13


def test_jitter_bounded_and_boundary_fixed():
    m = 16
    xy, tris, bnd, used, _ = fem.lshape(m)
    xj = fem.jitter_nodes(xy, ~bnd, 1.0 / m, seed=2)
    d = np.abs(xj - xy)
    assert d[bnd].max() == 0.0
    assert d.max() <= 0.2 / m
    assert d[~bnd & used].max() > 0.15 / m


def test_cube_checkerboard_and_kuhn_stencil():
    p = configs.cube(8)
    nnz = np.diff(p["rowptr"])
    assert nnz.max() == 15
    A = _mat(p, "A")
    d = A.diagonal()
    assert d.min() > 0 and abs(d.max() / d.min() - 1e3) < 1e-9
