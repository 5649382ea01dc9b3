"""Pins of the oracle's multicolour Gauss-Seidel smoother: the paper's
Gauss-Seidel smoothing (Section 4.1) with each level's rows visited colour by
colour.  The colouring is checked against its characterisation (a proper
colouring in which every vertex's colour is the first one free among its
earlier neighbours) and against closed forms on a path and a grid; the ordered
sweep against the textbook red-black sweep, the natural-order sweep, and the
invariants any Gauss-Seidel sweep in a colour order satisfies."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Oracle, amg, native
from workloads import configs
from tests.helpers import mats


def tridiag(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def random_spd(n, density, seed):
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=density, random_state=rng, format="csr")
    S = R + R.T
    S.data[:] = -np.abs(S.data)
    d = np.asarray(np.abs(S).sum(axis=1)).ravel() + 1.0
    return (S + sp.diags(d)).tocsr()


def edges(A):
    C = sp.coo_matrix(A)
    keep = (C.row != C.col) & (C.data != 0)
    i, j = C.row[keep], C.col[keep]
    return np.concatenate([i, j]), np.concatenate([j, i])  # both directions


def check_first_fit(A, colour):
    i, j = edges(A)
    assert np.all(colour[i] != colour[j]), "two neighbours share a colour"
    # every colour below c(i) appears among the neighbours j < i
    earlier = j < i
    pairs = np.unique(np.stack([i[earlier], colour[j[earlier]]], axis=1), axis=0)
    below = pairs[pairs[:, 1] < colour[pairs[:, 0]]]
    count = np.bincount(below[:, 0], minlength=A.shape[0])
    assert np.array_equal(count, colour), "a vertex skipped a free colour"


def test_colouring_of_a_path_and_a_grid():
    c, order = amg.colouring(tridiag(11))
    assert np.array_equal(c, np.arange(11) % 2)
    assert np.array_equal(order, np.r_[np.arange(0, 11, 2), np.arange(1, 11, 2)])
    m = 9  # 5-point Laplacian, natural (row-major) order: the checkerboard
    T = tridiag(m)
    A = sp.kron(sp.identity(m), T) + sp.kron(T, sp.identity(m))
    c, _ = amg.colouring(A.tocsr())
    ii, jj = np.meshgrid(np.arange(m), np.arange(m))
    assert np.array_equal(c, ((ii + jj) % 2).ravel())


@pytest.mark.parametrize("make", [
    lambda: random_spd(300, 0.02, 1),
    lambda: mats(configs.lshape(12, q=4, jitter_seed=3))[0],
    lambda: mats(configs.cube(6, q=4))[0],
])
def test_colouring_is_first_fit_on_every_level(make):
    A = make()
    o = Oracle(A, sp.identity(A.shape[0], format="csr"), q=2, qe=2, coarse_max=40, smoother="mcgs")
    for L in o.levels:
        check_first_fit(L.A, L.colour)
        assert L.colour.max() + 1 <= np.diff(L.A.indptr).max()  # at most max degree + 1
        assert np.all(np.diff(L.colour[L.order]) >= 0)
        for c in range(L.colour.max() + 1):
            assert np.all(np.diff(L.order[L.colour[L.order] == c]) > 0)


def test_ordered_sweep_reduces_to_natural_order():
    A = mats(configs.lshape(10, q=4, jitter_seed=2))[0]
    n = A.shape[0]
    rng = np.random.default_rng(4)
    b = rng.standard_normal((n, 3))
    x0 = rng.standard_normal((n, 3))
    ident = np.arange(n)
    for back in (False, True):
        a = native.gs_sweep(A, b, x0.copy(), backward=back)
        c = native.gs_sweep(A, b, x0.copy(), backward=back, order=ident)
        assert np.array_equal(a, c)
    a = native.gs_sweep(A, b, x0.copy(), backward=True)
    c = native.gs_sweep(A, b, x0.copy(), backward=False, order=ident[::-1])
    assert np.array_equal(a, c)


def test_red_black_sweeps_closed_form():
    """Path Laplacian tridiag(-1, 2, -1): the colour order is red-black, and a
    sweep is two vectorised half-steps."""
    n = 13
    A = tridiag(n)
    colour, order = amg.colouring(A)
    rng = np.random.default_rng(7)
    b = rng.standard_normal((n, 2))
    x0 = rng.standard_normal((n, 2))
    red, black = np.arange(0, n, 2), np.arange(1, n, 2)

    def half(x, rows):
        y = x.copy()
        pad = np.vstack([np.zeros((1, 2)), x, np.zeros((1, 2))])
        y[rows] = (b[rows] + pad[rows] + pad[rows + 2]) / 2.0
        return y

    fwd = half(half(x0, red), black)
    bwd = half(half(x0, black), red)
    assert np.allclose(native.gs_sweep(A, b, x0.copy(), order=order), fwd, rtol=0, atol=1e-14)
    assert np.allclose(native.gs_sweep(A, b, x0.copy(), backward=True, order=order), bwd, rtol=0, atol=1e-14)
    z = native.gs_sweep(A, b, np.zeros((n, 2)), order=order)
    assert np.allclose(z[red], b[red] / 2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_sweep_invariants(seed):
    """After a forward sweep in colour order the residual vanishes on the last
    colour (nothing changes those rows' neighbours afterwards); after a
    backward sweep on colour 0.  Reordering rows inside a colour changes
    nothing at all: rows of one colour never read each other."""
    A = mats(configs.lshape(14, q=4, jitter_seed=seed))[0]
    n = A.shape[0]
    colour, order = amg.colouring(A)
    assert colour.max() >= 2
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((n, 4))
    x0 = rng.standard_normal((n, 4))
    scale = np.abs(b).max() + np.abs(A).max() * np.abs(x0).max()
    x = native.gs_sweep(A, b, x0.copy(), order=order)
    last = colour == colour.max()
    assert np.abs((b - A @ x)[last]).max() < 1e-13 * scale
    assert np.abs((b - A @ x)[~last]).max() > 1e-3
    y = native.gs_sweep(A, b, x0.copy(), backward=True, order=order)
    assert np.abs((b - A @ y)[colour == 0]).max() < 1e-13 * scale
    shuffled = np.concatenate([rng.permutation(order[colour[order] == c]) for c in range(colour.max() + 1)])
    for back in (False, True):
        u = native.gs_sweep(A, b, x0.copy(), backward=back, order=order)
        v = native.gs_sweep(A, b, x0.copy(), backward=back, order=shuffled)
        assert np.array_equal(u, v)
