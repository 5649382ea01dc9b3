"""Build and load the oracle's plain-C loops (gcc, ctypes)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csrc", "oracle_loops.c")
LIB = os.path.join(_HERE, "csrc", "liboracle_loops.so")
_lib = None


def build(force=True):
    """Compile the oracle's C file with gcc (no GPU code involved)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        L.rs_first_pass.restype = ctypes.c_int64
        L.rs_first_pass.argtypes = [ctypes.c_int64, p, p, p, p, p]
        L.rs_second_pass.restype = ctypes.c_int64
        L.rs_second_pass.argtypes = [ctypes.c_int64, p, p, p]
        L.gs_sweep.restype = None
        L.gs_sweep.argtypes = [ctypes.c_int64, p, p, p, ctypes.c_int, p, p, ctypes.c_int, p]
        L.greedy_colour.restype = ctypes.c_int64
        L.greedy_colour.argtypes = [ctypes.c_int64, p, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def rs_first_pass(S, ST):
    """S, ST: scipy CSR strength matrices (row i = S_i, resp. S_i^T)."""
    n = S.shape[0]
    sp_, sc = np.ascontiguousarray(S.indptr, np.int64), np.ascontiguousarray(S.indices, np.int32)
    tp, tc = np.ascontiguousarray(ST.indptr, np.int64), np.ascontiguousarray(ST.indices, np.int32)
    cf = np.empty(n, dtype=np.int32)
    nc = lib().rs_first_pass(n, _ptr(sp_), _ptr(sc), _ptr(tp), _ptr(tc), _ptr(cf))
    if nc < 0:
        raise MemoryError("rs_first_pass")
    return cf


def rs_second_pass(S, cf):
    """Second pass on a first-pass splitting (returns a new array)."""
    cf = np.ascontiguousarray(cf, dtype=np.int32).copy()
    sp_, sc = np.ascontiguousarray(S.indptr, np.int64), np.ascontiguousarray(S.indices, np.int32)
    if lib().rs_second_pass(S.shape[0], _ptr(sp_), _ptr(sc), _ptr(cf)) < 0:
        raise MemoryError("rs_second_pass")
    return cf


def gs_sweep(A, b, x, backward=False, order=None):
    """In-place Gauss-Seidel sweep on x (n x q, C-contiguous float64), rows in
    natural order or in ``order`` (a permutation of 0..n-1); backward runs the
    sequence from its end."""
    n = A.shape[0]
    q = x.shape[1]
    assert x.flags.c_contiguous and x.dtype == np.float64
    bb = np.ascontiguousarray(b, dtype=np.float64)
    rp = np.ascontiguousarray(A.indptr, np.int64)
    ci = np.ascontiguousarray(A.indices, np.int32)
    va = np.ascontiguousarray(A.data, np.float64)
    od = None
    if order is not None:
        od = np.ascontiguousarray(order, np.int64)
        assert od.shape == (n,)
    lib().gs_sweep(n, _ptr(rp), _ptr(ci), _ptr(va), q, _ptr(bb), _ptr(x), 1 if backward else 0,
                   _ptr(od) if od is not None else None)
    return x


def greedy_colour(G):
    """First-fit colouring of the symmetric graph G (scipy CSR pattern, no
    diagonal) in the natural vertex order: (colour[n] int32, number of colours)."""
    n = G.shape[0]
    rp = np.ascontiguousarray(G.indptr, np.int64)
    ci = np.ascontiguousarray(G.indices, np.int32)
    colour = np.empty(n, dtype=np.int32)
    nc = lib().greedy_colour(n, _ptr(rp), _ptr(ci), _ptr(colour))
    if nc < 0:
        raise MemoryError("greedy_colour")
    return colour, int(nc)
