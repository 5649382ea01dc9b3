"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host setup (an implementation independent of the oracle's) builds the same
hierarchy.  No device call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1503_08462_amd as ae
from oracle import Oracle
from workloads import configs
from tests.helpers import mats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "amg_eig.h")).read()
    declared = set(re.findall(r"\b(amg_eig_[a-z_]+)\s*\(", hdr))
    assert declared == set(ae.EXPORTED)
    lib = ctypes.CDLL(ae.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("make,cm", [
    (lambda: configs.config(0), 130),
    (lambda: configs.lshape(24, q=10, jitter_seed=2), 300),
    (lambda: configs.cube(12, q=8), 100),
    (lambda: configs.oscillator(40, q=10), 150),
    (lambda: configs.quadrants(16, q=6), 100),
])
def test_setup_matches_oracle(make, cm):
    p = make()
    A, M = mats(p)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=cm, qe=12))
    info = ctx.info()
    o = Oracle(A, M, q=p["q"], qe=12, coarse_max=cm, coarse_min=26)
    assert info["dims"].tolist() == [L.n for L in o.levels]
    for l in range(info["levels"] - 1):
        assert np.array_equal(ctx.splitting(l), o.levels[l].cf)
        rp, ci, pv = ctx.prolongation(l)
        P = sp.csr_matrix((pv, ci, rp), shape=(info["dims"][l], info["dims"][l + 1]))
        assert abs(P - o.levels[l].P).max() <= 1e-14
        rp, ci, a, m = ctx.level_matrix(l + 1)
        Al, Ml = sp.csr_matrix((a, ci, rp)), sp.csr_matrix((m, ci, rp))
        assert abs(Al - o.levels[l + 1].A).max() <= 1e-13 * abs(o.levels[l + 1].A).max()
        assert abs(Ml - o.levels[l + 1].M).max() <= 1e-13 * abs(o.levels[l + 1].M).max()
    lam = ctx.coarse_eigenvalues()
    # dense symmetric eigensolvers are backward stable: errors of order eps * ||A_n||
    assert np.abs(lam - o.lam_n).max() <= 1e-12 * np.abs(o.lam_n).max()
    ctx.close()


@pytest.mark.parametrize("make,cm", [
    (lambda: configs.lshape(24, q=10, jitter_seed=2), 300),
    (lambda: configs.cube(12, q=8), 100),
    (lambda: configs.oscillator(40, q=10), 150),
])
def test_colouring_matches_oracle(make, cm):
    """Multicolour Gauss-Seidel: the library's first-fit colouring of every
    smoothed level equals the oracle's, row for row."""
    p = make()
    A, M = mats(p)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"],
                     ae.defaults(coarse_max=cm, qe=12, smoother=ae.SMOOTH_GAUSS_SEIDEL))
    o = Oracle(A, M, q=p["q"], qe=12, coarse_max=cm, coarse_min=26, smoother="mcgs")
    info = ctx.info()
    assert info["dims"].tolist() == [L.n for L in o.levels]
    for l in range(info["levels"] - 1):
        colour, nc = ctx.colouring(l)
        assert np.array_equal(colour, o.levels[l].colour), l
        assert nc == o.levels[l].colour.max() + 1
    with pytest.raises(ae.AmgEigError):
        ctx.colouring(info["levels"] - 1)
    ctx.close()
    plain = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarse_max=cm, qe=12))
    with pytest.raises(ae.AmgEigError):
        plain.colouring(0)
    plain.close()


def test_shift_options():
    """Remark 3.1 shift: rejected unless below the coarsest level's smallest
    eigenvalue; with multicolour Gauss-Seidel the colouring follows the
    shifted operator's pattern, as the oracle's does."""
    p = configs.oscillator(40, q=6)
    A, M = mats(p)
    o0 = Oracle(A, M, q=6, qe=8, coarse_max=150, coarse_min=26)
    lam1 = o0.lam_n[0]
    for kw in (dict(shift=1.001 * lam1), dict(shift=float("nan")), dict(shift=float("inf"))):
        with pytest.raises(ae.AmgEigError) as e:
            ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 6, ae.defaults(coarse_max=150, qe=8, **kw))
        assert e.value.code == ae.EINVAL, kw
    sigma = 0.9 * lam1
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 6,
                     ae.defaults(coarse_max=150, qe=8, shift=sigma, smoother=ae.SMOOTH_GAUSS_SEIDEL))
    o = Oracle(A, M, q=6, qe=8, coarse_max=150, coarse_min=26, smoother="mcgs", shift=sigma)
    for l in range(ctx.info()["levels"] - 1):
        assert np.array_equal(ctx.colouring(l)[0], o.levels[l].colour)
    ctx.close()


def test_guard_rule_and_width_rounding():
    """Block width = guard rule on the coarsest eigenvalues (no block ending
    inside a relative gap < 1e-2), rounded up to a multiple of 4."""
    from oracle import guard_count
    for p, q in ((configs.square(32, q=2), 2), (configs.oscillator(64, q=6), 6), (configs.cube(12, q=5), 5)):
        ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], q, ae.defaults(coarse_max=200))
        lam = ctx.coarse_eigenvalues()
        want = guard_count(lam, q)
        assert ctx.info()["qe"] == (want + 3) // 4 * 4
        ctx.close()


@pytest.mark.parametrize("mutate,code", [
    ("unsorted", ae.EINVAL), ("range", ae.EINVAL), ("negdiag", ae.ENOTSPD), ("rowptr", ae.EINVAL),
    ("q0", ae.EINVAL), ("toowide", ae.EINVAL), ("nan", ae.EINVAL), ("chebdeg3", ae.EINVAL), ("nu2", ae.EINVAL),
])
def test_validation_errors(mutate, code):
    p = configs.square(8, q=2)
    rp, col, a, m = p["rowptr"].copy(), p["col"].copy(), p["A"].copy(), p["M"].copy()
    q = 2
    opts = ae.defaults(coarse_max=20, coarse_min=8)
    if mutate == "unsorted":
        col[1], col[2] = col[2], col[1]
    elif mutate == "range":
        col[3] = 10 ** 6
    elif mutate == "negdiag":
        a[0] = -1.0
    elif mutate == "rowptr":
        rp[5] = rp[4] - 1
    elif mutate == "q0":
        q = 0
    elif mutate == "toowide":
        opts.qe = 200
    elif mutate == "nan":
        m[7] = np.nan
    elif mutate == "chebdeg3":  # the device smoother implements degree 2 only
        opts.smoother, opts.cheb_degree = ae.SMOOTH_CHEBYSHEV, 3
    elif mutate == "nu2":
        opts.nu_pre = 2
    with pytest.raises(ae.AmgEigError) as ei:
        ae.Context(rp, col, a, m, q, opts)
    assert ei.value.code == code


def test_chebyshev_degree_two_is_accepted():
    p = configs.square(8, q=2)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 2,
                     ae.defaults(coarse_max=20, coarse_min=8, smoother=ae.SMOOTH_CHEBYSHEV, cheb_degree=2))
    assert ctx.info()["qe"] >= 2
    ctx.close()


def test_calls_out_of_order_are_rejected_on_the_host():
    p = configs.square(8, q=2)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 2, ae.defaults(coarse_max=20, coarse_min=8))
    with pytest.raises(ae.AmgEigError) as ei:
        ctx.correct(1)
    assert ei.value.code == ae.ESTATE
    with pytest.raises(ae.AmgEigError) as ei:
        ctx.init()
    assert ei.value.code == ae.ESTATE
    ctx.close()


def test_joint_batch_calls_reject_unbound_members_on_the_host():
    """The joint batch entry points check their members before any device
    call: unbound (or uninitialised) members are state errors, and an empty
    list is a no-op."""
    p = configs.square(8, q=2)
    ctx = ae.Context(p["rowptr"], p["col"], p["A"], p["M"], 2, ae.defaults(coarse_max=20, coarse_min=8))
    for call in (lambda: ae.init_batch_joint([ctx]), lambda: ae.correct_batch_joint([ctx], 1)):
        with pytest.raises(ae.AmgEigError) as ei:
            call()
        assert ei.value.code == ae.ESTATE
    ae.init_batch_joint([])
    ae.correct_batch_joint([], 1)
    ctx.close()


def test_setup_rejects_unknown_coarsening_without_device():
    """coarsening accepts only the host Ruge-Stueben passes (0, the default)
    and the device PMIS setup (1); another value is refused before any device
    call."""
    p = configs.config(0)
    o = ae.defaults()
    assert o.coarsening == ae.COARSEN_RS and o.coarsen_seed == 0
    with pytest.raises(ae.AmgEigError) as e:
        ae.Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], ae.defaults(coarsening=5))
    assert e.value.code == ae.EINVAL


def test_device_setup_entry_points_check_arguments_on_the_host():
    """The device setup calls refuse malformed sizes and missing arrays before
    any device work, and accept empty problems without touching the device."""
    lib = ae._lib
    nnz, nc = ctypes.c_int64(), ctypes.c_int64()
    rounds = ctypes.c_int(-1)
    assert lib.amg_eig_galerkin(-1, 0, *([None] * 14), 0, ctypes.byref(nnz), None) == ae.EINVAL
    assert lib.amg_eig_galerkin(4, 2, *([None] * 14), 0, ctypes.byref(nnz), None) == ae.EINVAL
    assert lib.amg_eig_strength(-1, None, None, None, 0.25, None, None) == ae.EINVAL
    assert lib.amg_eig_strength(0, None, None, None, 0.25, None, None) == ae.OK
    assert lib.amg_eig_strength(3, None, None, None, 0.25, None, None) == ae.EINVAL
    assert lib.amg_eig_pmis(-1, None, None, None, None, 1, None, ctypes.byref(rounds), None) == ae.EINVAL
    assert lib.amg_eig_pmis(0, None, None, None, None, 1, None, ctypes.byref(rounds), None) == ae.OK
    assert rounds.value == 0
    assert lib.amg_eig_pmis(5, None, None, None, None, 0, None, ctypes.byref(rounds), None) == ae.EINVAL
    assert lib.amg_eig_interpolation(-1, *([None] * 8), 0, ctypes.byref(nnz), ctypes.byref(nc), None) == ae.EINVAL
    assert lib.amg_eig_interpolation(3, *([None] * 8), 0, ctypes.byref(nnz), ctypes.byref(nc), None) == ae.EINVAL
    assert lib.amg_eig_transpose(-1, 0, *([None] * 6), None) == ae.EINVAL
    assert lib.amg_eig_transpose(2, 2, *([None] * 6), None) == ae.EINVAL
    for n in (0, 4097):
        assert lib.amg_eig_dense_sygv(n, *([None] * 5), None) == ae.EINVAL


def test_options_struct_layout_matches_the_binding(tmp_path):
    """The ctypes mirrors of amg_eig_opts and amg_eig_csr have the C structs'
    sizes and field offsets (a C program built with gcc against
    include/amg_eig.h prints them), so they cross the boundary intact."""
    import subprocess
    fields = [f[0] for f in ae.Opts._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"amg_eig.h\"\nint main(void) {\n"
                   "  printf(\"size %zu\\n\", sizeof(amg_eig_opts));\n"
                   + "".join("  printf(\"%s %%zu\\n\", offsetof(amg_eig_opts, %s));\n" % (f, f) for f in fields)
                   + "  printf(\"csr_size %zu\\n\", sizeof(amg_eig_csr));\n"
                   + "".join("  printf(\"csr_%s %%zu\\n\", offsetof(amg_eig_csr, %s));\n" % (f, f)
                             for f, _ in ae.Csr._fields_)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(ae.Opts)
    for f in fields:
        assert int(out[f]) == getattr(ae.Opts, f).offset, f
    assert int(out["csr_size"]) == ctypes.sizeof(ae.Csr)
    for f, _ in ae.Csr._fields_:
        assert int(out["csr_" + f]) == getattr(ae.Csr, f).offset, f


def test_product_path_never_reaches_the_oracle():
    """The package (binding, autotuner, serving loop, HIP and C++ sources)
    names no module or file of the oracle, and importing it leaves the oracle
    unloaded: every step of a solve runs in libamg_eig.so."""
    import subprocess
    import sys
    pkg = os.path.join(ROOT, "paper_1503_08462_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), f
                assert "liboracle" not in text and "oracle/csrc" not in text, f
    code = "import sys; import paper_1503_08462_amd; print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))"
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "False"
