"""Device Galerkin products (Section 2, eq. (2.5)) through the C ABI: every
coarse level of the hierarchy formed on the GPU from the host's prolongations
equals the host setup's level bit for bit (same accumulation order), and equals
the definition P^T A P formed by SciPy (the oracle's Galerkin step) within
rounding; the whole chain of levels formed on the device from the device's own
previous level; edge cases (empty coarse space, an output capacity too small)."""
import ctypes
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1503_08462_amd as ae
from oracle.amg import galerkin as oracle_galerkin
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a, dt):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()


def _levels(p, cm):
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=cm, qe=12))
    info = ctx.info()
    dims = [int(d) for d in info["dims"]]
    mats = [ctx.level_matrix(l) for l in range(len(dims))]
    pro = []
    for l in range(len(dims) - 1):
        rp, ci, pv = ctx.prolongation(l)
        P = sp.csr_matrix((pv, ci, rp), shape=(dims[l], dims[l + 1]))
        Pt = P.T.tocsr()
        Pt.sort_indices()
        pro.append((P, Pt))
    ctx.close()
    return dims, mats, pro


def _device_galerkin(torch, n, nc, level, P, Pt):
    rp, ci, a, m = level
    args = [_dev(torch, rp, np.int64), _dev(torch, ci, np.int32), _dev(torch, a, np.float64),
            _dev(torch, m, np.float64), _dev(torch, P.indptr, np.int64), _dev(torch, P.indices, np.int32),
            _dev(torch, P.data, np.float64), _dev(torch, Pt.indptr, np.int64), _dev(torch, Pt.indices, np.int32),
            _dev(torch, Pt.data, np.float64)]
    out = ae.galerkin(n, nc, *args)
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in out)


CASES = [
    ("square64", lambda: configs.square(64, q=4), 130),
    ("lshape24j", lambda: configs.lshape(24, q=10, jitter_seed=2), 300),
    ("cube12", lambda: configs.cube(12, q=8), 100),
    ("cube20", lambda: configs.cube(20, q=8), 200),
    ("oscillator40", lambda: configs.oscillator(40, q=10), 150),
    ("quadrants16", lambda: configs.quadrants(16, q=6), 100),
]


@pytest.mark.parametrize("name,make,cm", CASES, ids=[c[0] for c in CASES])
def test_galerkin_levels_match_host_and_definition(name, make, cm):
    import torch
    p = make()
    dims, mats, pro = _levels(p, cm)
    for l in range(len(dims) - 1):
        _say("galerkin %s level %d -> %d (%d -> %d rows)" % (name, l, l + 1, dims[l], dims[l + 1]))
        P, Pt = pro[l]
        cp, cc, ca, cmv = _device_galerkin(torch, dims[l], dims[l + 1], mats[l], P, Pt)
        hp, hc, ha, hm = mats[l + 1]
        # the host setup's level, bit for bit
        assert np.array_equal(cp, hp) and np.array_equal(cc, hc)
        assert np.array_equal(ca, ha) and np.array_equal(cmv, hm)
        # the definition, formed by SciPy (another summation order)
        rp, ci, a, m = mats[l]
        A = sp.csr_matrix((a, ci, rp), shape=(dims[l], dims[l]))
        M = sp.csr_matrix((m, ci, rp), shape=(dims[l], dims[l]))
        for vals, X in ((ca, A), (cmv, M)):
            C = sp.csr_matrix((vals, cc, cp), shape=(dims[l + 1], dims[l + 1]))
            ref = oracle_galerkin(P, X)
            scale = abs(ref).max()
            assert abs(C - ref).max() <= 1e-13 * scale


def test_galerkin_chain_on_device():
    """Each coarse level formed from the device's own previous level (the host
    provides only the prolongations): the chain ends on the host's coarsest
    level, bit for bit."""
    import torch
    p = configs.oscillator(200, q=10)
    dims, mats, pro = _levels(p, 300)
    _say("galerkin chain oscillator200: %s" % dims)
    cur = mats[0]
    t0 = time.perf_counter()
    for l in range(len(dims) - 1):
        P, Pt = pro[l]
        cur = _device_galerkin(torch, dims[l], dims[l + 1], cur, P, Pt)
        for x, y in zip(cur, mats[l + 1]):
            assert np.array_equal(x, y), "level %d" % (l + 1)
    _say("chain of %d levels on the device: %.1f ms with transfers" % (len(dims) - 1,
                                                                       1e3 * (time.perf_counter() - t0)))


def _raw(torch, n, nc, level, P, Pt, c_ptr, cap, outs):
    keep = [_dev(torch, x, dt) for x, dt in (
        (level[0], np.int64), (level[1], np.int32), (level[2], np.float64), (level[3], np.float64),
        (P.indptr, np.int64), (P.indices, np.int32), (P.data, np.float64),
        (Pt.indptr, np.int64), (Pt.indices, np.int32), (Pt.data, np.float64))]
    nnz = ctypes.c_int64(-1)
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in keep]
    o = [ctypes.c_void_p(t.data_ptr()) if t is not None else None for t in outs]
    rc = ae._lib.amg_eig_galerkin(n, nc, *ptrs, ctypes.c_void_p(c_ptr.data_ptr()), *o, cap, ctypes.byref(nnz),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, nnz.value


def test_galerkin_capacity_and_empty():
    import torch
    p = configs.square(32, q=4)
    dims, mats, pro = _levels(p, 100)
    P, Pt = pro[0]
    n, nc = dims[0], dims[1]
    want = mats[1]
    _say("galerkin capacity square32: %d -> %d" % (n, nc))
    c_ptr = torch.full((nc + 1,), -7, dtype=torch.int64, device="cuda")
    rc, nnz = _raw(torch, n, nc, mats[0], P, Pt, c_ptr, 0, (None, None, None))
    assert rc == ae.EWORKSPACE and nnz == want[0][-1]
    assert np.array_equal(c_ptr.cpu().numpy(), want[0])
    small = nnz - 1
    outs = (torch.zeros(small, dtype=torch.int32, device="cuda"), torch.zeros(small, dtype=torch.float64, device="cuda"),
            torch.zeros(small, dtype=torch.float64, device="cuda"))
    rc, nnz2 = _raw(torch, n, nc, mats[0], P, Pt, c_ptr, small, outs)
    assert rc == ae.EWORKSPACE and nnz2 == nnz
    assert not outs[0].any().item() and not outs[1].any().item()
    # exact capacity
    outs = (torch.zeros(nnz, dtype=torch.int32, device="cuda"), torch.zeros(nnz, dtype=torch.float64, device="cuda"),
            torch.zeros(nnz, dtype=torch.float64, device="cuda"))
    rc, nnz3 = _raw(torch, n, nc, mats[0], P, Pt, c_ptr, nnz, outs)
    assert rc == ae.OK and nnz3 == nnz
    assert np.array_equal(outs[0].cpu().numpy(), want[1]) and np.array_equal(outs[1].cpu().numpy(), want[2])
    # an empty coarse space: P with no columns
    _say("galerkin empty coarse space")
    P0 = sp.csr_matrix((n, 0))
    Pt0 = sp.csr_matrix((0, n))
    c0 = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    rc, nnz0 = _raw(torch, n, 0, mats[0], P0, Pt0, c0, 0, (None, None, None))
    assert rc == ae.OK and nnz0 == 0 and c0.item() == 0
    # malformed: negative size
    rc, _ = _raw(torch, -1, nc, mats[0], P, Pt, c_ptr, 0, (None, None, None))
    assert rc == ae.EINVAL
