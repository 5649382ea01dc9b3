"""The row-parallel setup steps of Section 2 on the device, through the C ABI:
strong couplings (eq. (2.1)), direct interpolation from a C/F splitting (eqs.
(2.2)-(2.4)) and the transpose of P, chained level by level with the device
Galerkin products (eq. (2.5)), each level starting from the device's own
previous level.  Only the C/F splitting comes from the host (the library's
Ruge-Stueben passes, read through its inspector).  Every device result equals
the host setup's bit for bit, the strong couplings equal the oracle's eq.
(2.1) exactly, and P equals the oracle's direct interpolation within rounding;
edge cases: an all-F splitting, too small an output capacity, bad arguments."""
import ctypes
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1503_08462_amd as ae
from oracle.amg import direct_interpolation, strength
from workloads import configs

pytestmark = pytest.mark.gpu

THETA = 0.25


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()


def _host(ctx):
    dims = [int(d) for d in ctx.info()["dims"]]
    mats = [ctx.level_matrix(l) for l in range(len(dims))]
    cfs = [ctx.splitting(l) for l in range(len(dims) - 1)]
    pros = [ctx.prolongation(l) for l in range(len(dims) - 1)]
    return dims, mats, cfs, pros


CASES = [
    ("square64", lambda: configs.square(64, q=4), 130),
    ("lshape24j", lambda: configs.lshape(24, q=10, jitter_seed=2), 300),
    ("cube20", lambda: configs.cube(20, q=8), 200),
    ("oscillator200", lambda: configs.oscillator(200, q=10), 300),
    ("quadrants16", lambda: configs.quadrants(16, q=6), 100),
]


@pytest.mark.parametrize("name,make,cm", CASES, ids=[c[0] for c in CASES])
def test_setup_chain_on_device(name, make, cm):
    import torch
    p = make()
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=cm, qe=12, theta=THETA))
    dims, mats, cfs, pros = _host(ctx)
    ctx.close()
    rp, ci, a, m = mats[0]
    x = [_dev(torch, rp, np.int64), _dev(torch, ci, np.int32), _dev(torch, a, np.float64), _dev(torch, m, np.float64)]
    for l in range(len(dims) - 1):
        n = dims[l]
        _say("setup %s level %d (%d rows)" % (name, l, n))
        # eq. (2.1)
        strong = ae.strength(x[0], x[1], x[2], THETA)
        torch.cuda.synchronize()
        hp, hc, ha, hm = (t.cpu().numpy() for t in x)
        A = sp.csr_matrix((ha, hc, hp), shape=(n, n))
        S = strength(A, THETA)
        s_host = strong.cpu().numpy().astype(bool)
        rows = np.repeat(np.arange(n), np.diff(hp))
        Sd = sp.csr_matrix((np.ones(int(s_host.sum())), (rows[s_host], hc[s_host])), shape=(n, n))
        Sd.sort_indices()
        assert np.array_equal(Sd.indptr, S.indptr) and np.array_equal(Sd.indices, S.indices)
        # eqs. (2.2)-(2.4) from the host's C/F splitting
        cf = _dev(torch, cfs[l], np.int32)
        p_ptr, p_col, p_val, nc = ae.interpolation(x[0], x[1], x[2], strong, cf)
        torch.cuda.synchronize()
        assert nc == dims[l + 1]
        want = pros[l]
        got = (p_ptr.cpu().numpy(), p_col.cpu().numpy(), p_val.cpu().numpy())
        for g, w in zip(got, want):
            assert np.array_equal(g, w)
        P = sp.csr_matrix((got[2], got[1], got[0]), shape=(n, nc))
        Pref = direct_interpolation(A, S, cfs[l].astype(np.int64))
        assert abs(P - Pref).max() <= 1e-14 * max(1.0, abs(Pref).max())
        # transpose
        pt = ae.transpose(p_ptr, p_col, p_val, nc)
        torch.cuda.synchronize()
        Pt = P.T.tocsr()
        Pt.sort_indices()
        assert np.array_equal(pt[0].cpu().numpy(), Pt.indptr)
        assert np.array_equal(pt[1].cpu().numpy(), Pt.indices)
        assert np.array_equal(pt[2].cpu().numpy(), Pt.data)
        # eq. (2.5) from the device's own P and P^T
        x = list(ae.galerkin(n, nc, *x, p_ptr, p_col, p_val, *pt))
        torch.cuda.synchronize()
        for g, w in zip(x, mats[l + 1]):
            assert np.array_equal(g.cpu().numpy(), w), "level %d" % (l + 1)


def test_interpolation_edges():
    import torch
    p = configs.square(32, q=4)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=100, qe=8))
    dims, mats, cfs, pros = _host(ctx)
    ctx.close()
    rp, ci, a, _ = mats[0]
    n = dims[0]
    x = [_dev(torch, rp, np.int64), _dev(torch, ci, np.int32), _dev(torch, a, np.float64)]
    strong = ae.strength(*x, THETA)
    s = torch.cuda.current_stream().cuda_stream
    # all F: every row empty, no columns
    _say("interpolation all-F square32")
    cf0 = torch.zeros(n, dtype=torch.int32, device="cuda")
    p_ptr, p_col, p_val, nc = ae.interpolation(*x, strong, cf0)
    torch.cuda.synchronize()
    assert nc == 0 and p_col.numel() == 0 and not p_ptr.any().item()
    pt = ae.transpose(p_ptr, p_col, p_val, 0)
    torch.cuda.synchronize()
    assert pt[0].numel() == 1 and pt[0].item() == 0
    # too small a capacity: p_ptr, nnz and nc reported, EWORKSPACE
    _say("interpolation capacity square32")
    cf = _dev(torch, cfs[0], np.int32)
    p_ptr = torch.full((n + 1,), -3, dtype=torch.int64, device="cuda")
    small = int(pros[0][0][-1]) - 1
    col = torch.zeros(small, dtype=torch.int32, device="cuda")
    val = torch.zeros(small, dtype=torch.float64, device="cuda")
    nnz, ncv = ctypes.c_int64(), ctypes.c_int64()
    rc = ae._lib.amg_eig_interpolation(n, *[ctypes.c_void_p(t.data_ptr()) for t in x + [strong, cf, p_ptr, col, val]],
                                       small, ctypes.byref(nnz), ctypes.byref(ncv), ctypes.c_void_p(s))
    torch.cuda.synchronize()
    assert rc == ae.EWORKSPACE and nnz.value == small + 1 and ncv.value == dims[1]
    assert np.array_equal(p_ptr.cpu().numpy(), pros[0][0]) and not col.any().item()
    # bad arguments are refused on the host
    assert ae._lib.amg_eig_strength(n, ctypes.c_void_p(x[0].data_ptr()), None, None, 1.5, None,
                                    ctypes.c_void_p(s)) == ae.EINVAL
    assert ae._lib.amg_eig_transpose(-1, 0, None, None, None, None, None, None, ctypes.c_void_p(s)) == ae.EINVAL


def _device_hierarchy(torch, x, n, seed, coarse_max, theta=THETA, check=None, second_pass=False):
    """Levels built on the device only: strength, PMIS, interpolation,
    transpose, Galerkin, until n <= coarse_max or coarsening stalls.  check(l,
    x, strong, cf, P, Pt, xnext) is called per level with device tensors."""
    from workloads.prng import uniform01
    dims = [n]
    rounds = []
    l = 0
    while n > coarse_max:
        strong = ae.strength(x[0], x[1], x[2], theta)
        rnd = _dev(torch, uniform01(seed + l, np.arange(n)), np.float64)
        cf, r = ae.pmis(x[0], x[1], strong, rnd, second_pass=second_pass)
        p_ptr, p_col, p_val, nc = ae.interpolation(x[0], x[1], x[2], strong, cf)
        if nc == 0 or nc > 0.9 * n:
            break
        pt = ae.transpose(p_ptr, p_col, p_val, nc)
        xn = list(ae.galerkin(n, nc, *x, p_ptr, p_col, p_val, *pt))
        if check is not None:
            check(l, x, strong, rnd, cf, (p_ptr, p_col, p_val, nc), pt, xn)
        x, n = xn, nc
        dims.append(n)
        rounds.append(r)
        l += 1
    return dims, rounds


PMIS_CASES = [
    ("square48", lambda: configs.square(48, q=4)),
    ("lshape24j", lambda: configs.lshape(24, q=10, jitter_seed=2)),
    ("cube16", lambda: configs.cube(16, q=8)),
    ("oscillator100", lambda: configs.oscillator(100, q=10)),
    ("quadrants16", lambda: configs.quadrants(16, q=6)),
]


@pytest.mark.parametrize("second_pass", [False, True], ids=["pmis", "pmis2"])
@pytest.mark.parametrize("name,make", PMIS_CASES, ids=[c[0] for c in PMIS_CASES])
def test_pmis_hierarchy_on_device_matches_oracle(name, make, second_pass):
    """The whole hierarchy built on the device (PMIS in place of the host's
    Ruge-Stueben passes); each level's steps against the oracle's on the same
    input: strength and the splitting exactly, P within rounding, the Galerkin
    operators within rounding of P^T A P."""
    import torch
    from oracle.amg import galerkin, pmis_splitting
    p = make()
    n = p["n"]

    def check(l, x, strong, rnd, cf, P, pt, xn):
        hp, hc, ha, hm = (t.cpu().numpy() for t in x)
        nn = hp.size - 1
        A = sp.csr_matrix((ha, hc, hp), shape=(nn, nn))
        M = sp.csr_matrix((hm, hc, hp), shape=(nn, nn))
        cf_o, S, rounds_o = pmis_splitting(A, rnd.cpu().numpy(), THETA, second_pass=second_pass)
        cf_d = cf.cpu().numpy()
        _say("pmis %s level %d: %d rows, %d C, %d rounds" % (name, l, nn, int(cf_d.sum()), rounds_o))
        assert np.array_equal(cf_d, cf_o)
        Pd = sp.csr_matrix((P[2].cpu().numpy(), P[1].cpu().numpy(), P[0].cpu().numpy()), shape=(nn, P[3]))
        Po = direct_interpolation(A, S, cf_o)
        assert Pd.shape == Po.shape and abs(Pd - Po).max() <= 1e-14 * max(1.0, abs(Po).max())
        cp, cc, ca, cm = (t.cpu().numpy() for t in xn)
        for vals, X in ((ca, A), (cm, M)):
            C = sp.csr_matrix((vals, cc, cp), shape=(P[3], P[3]))
            ref = galerkin(Pd, X)
            assert abs(C - ref).max() <= 1e-13 * abs(ref).max()

    x = [_dev(torch, p["rowptr"], np.int64), _dev(torch, p["col"], np.int32), _dev(torch, p["A"], np.float64),
         _dev(torch, p["M"], np.float64)]
    dims, rounds = _device_hierarchy(torch, x, n, 1000, 120, check=check, second_pass=second_pass)
    _say("pmis %s: levels %s, rounds %s" % (name, dims, rounds))
    assert len(dims) >= 3


def test_device_setup_time_oscillator1024():
    """Setup of the 1,046,529-row oscillator: the whole hierarchy on the device
    (PMIS splitting) beside the host setup (Ruge-Stueben), timed; properties
    only (every point decided, each level smaller than the last)."""
    import time
    import torch
    p = configs.oscillator(1024, q=16)
    n = p["n"]
    _say("device setup oscillator1024: %d rows" % n)
    x = [_dev(torch, p["rowptr"], np.int64), _dev(torch, p["col"], np.int32), _dev(torch, p["A"], np.float64),
         _dev(torch, p["M"], np.float64)]
    torch.cuda.synchronize()

    def check(l, x, strong, rnd, cf, P, pt, xn):
        c = cf.cpu().numpy()
        assert set(np.unique(c).tolist()) <= {0, 1}

    _device_hierarchy(torch, x, n, 1000, 512)  # warm-up (module load)
    t0 = time.perf_counter()
    dims, rounds = _device_hierarchy(torch, x, n, 1000, 512)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    dims2, rounds2 = _device_hierarchy(torch, x, n, 1000, 512, second_pass=True)
    torch.cuda.synchronize()
    t_dev2 = time.perf_counter() - t0
    _say("device setup (PMIS with the second pass) %.1f ms, levels %s" % (1e3 * t_dev2, dims2))
    _device_hierarchy(torch, x, n, 1000, 512, check=check)
    assert all(a > b for a, b in zip(dims, dims[1:]))
    t0 = time.perf_counter()
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(qe=24))
    t_host = time.perf_counter() - t0
    hd = [int(d) for d in ctx.info()["dims"]]
    ctx.close()
    _say("device setup (PMIS) %.1f ms, levels %s, rounds %s; host setup (RS, with the coarsest "
         "eigen-decomposition) %.1f ms, levels %s" % (1e3 * t_dev, dims, rounds, 1e3 * t_host, hd))
