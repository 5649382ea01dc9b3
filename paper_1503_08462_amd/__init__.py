"""Python binding of the amg_eig C ABI (include/amg_eig.h).

Argument marshalling only: every step of the solver runs in the HIP library
libamg_eig.so built from csrc/ for gfx950.  PyTorch supplies the device
workspace (a uint8 tensor of `footprint()` bytes) and the HIP stream.  There is
no fallback: if the library is missing, importing this package raises.
"""
import ctypes
import os

import numpy as np

# PyTorch ships its own HIP runtime (same soname as /opt/rocm's).  Loading torch
# first makes this library bind to that already-loaded runtime, so the process
# holds a single HIP runtime that both torch (memory, streams) and the kernels use.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamg_eig.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libamg_eig.so is not built; run `python paper_1503_08462_amd/build.py` "
                      "(hipcc for gfx950). There is no CPU fallback.")

_lib = ctypes.CDLL(LIB_PATH)

OK, NOT_CONVERGED, WIDENED = 0, 1, 2
EINVAL, ENOTSPD, EBREAKDOWN, ENOMEM, EWORKSPACE, EHIP, ECANCELLED, ESTATE = -1, -2, -3, -4, -5, -6, -7, -8
SMOOTH_L1JACOBI, SMOOTH_CHEBYSHEV, SMOOTH_GAUSS_SEIDEL = 0, 1, 2
COARSEN_RS, COARSEN_PMIS = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
INIT_NESTED, INIT_RANDOM, INIT_USER = 0, 1, 2

EXPORTED = [
    "amg_eig_opts_default", "amg_eig_setup", "amg_eig_footprint", "amg_eig_bind", "amg_eig_init",
    "amg_eig_correct", "amg_eig_progress", "amg_eig_solve", "amg_eig_correct_batch", "amg_eig_correct_batch_joint",
    "amg_eig_init_batch_joint", "amg_eig_info",
    "amg_eig_level_matrix", "amg_eig_level_prolongation", "amg_eig_level_splitting", "amg_eig_level_colouring",
    "amg_eig_coarse_eigenvalues", "amg_eig_iterate", "amg_eig_destroy", "amg_eig_strerror",
    "amg_eig_last_error", "amg_eig_timing", "amg_eig_site_stats", "amg_eig_set_cpt", "amg_eig_get_cpt",
    "amg_eig_tune_time", "amg_eig_bind_static", "amg_eig_galerkin",
    "amg_eig_strength", "amg_eig_interpolation", "amg_eig_transpose", "amg_eig_pmis",
    "amg_eig_dense_sygv",
]
TUNE_VCYCLE, TUNE_FP64, TUNE_FP64_WIDE = 0, 1, 2
SITES = ["residual", "presmooth", "postsmooth", "dualspmm", "gram", "restrict", "final", "small"]


class Opts(ctypes.Structure):
    _fields_ = [
        ("theta", ctypes.c_double), ("coarse_max", ctypes.c_int), ("coarse_min", ctypes.c_int),
        ("max_levels", ctypes.c_int), ("qe", ctypes.c_int), ("guard_gap", ctypes.c_double),
        ("smoother", ctypes.c_int), ("cheb_degree", ctypes.c_int), ("cheb_lo", ctypes.c_double),
        ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("precision", ctypes.c_int),
        ("tol", ctypes.c_double), ("max_steps", ctypes.c_int), ("use_graph", ctypes.c_int),
        ("qe_max", ctypes.c_int),
        ("shift", ctypes.c_double),
        ("coarsening", ctypes.c_int), ("coarsen_seed", ctypes.c_uint64),
        ("vcycles", ctypes.c_int),
    ]


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


_vp, _i, _i64, _d, _u64, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_size_t
_sig = {
    "amg_eig_opts_default": (None, [_vp]),
    "amg_eig_setup": (_i, [_vp, _vp, _i, _vp, _vp]),
    "amg_eig_footprint": (_i, [_vp, _vp]),
    "amg_eig_bind": (_i, [_vp, _vp, _sz, _vp]),
    "amg_eig_bind_static": (_i, [_vp, _vp, _vp]),
    "amg_eig_init": (_i, [_vp, _i, _u64, _vp, _i64]),
    "amg_eig_correct": (_i, [_vp, _i]),
    "amg_eig_progress": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "amg_eig_solve": (_i, [_vp, _d, _i, _vp, _vp, _i64]),
    "amg_eig_correct_batch": (_i, [_vp, _i, _i, _vp]),
    "amg_eig_correct_batch_joint": (_i, [_vp, _i, _i]),
    "amg_eig_init_batch_joint": (_i, [_vp, _i]),
    "amg_eig_info": (_i, [_vp, _vp, _vp, _vp]),
    "amg_eig_level_matrix": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
    "amg_eig_level_prolongation": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "amg_eig_level_splitting": (_i, [_vp, _i, _vp]),
    "amg_eig_level_colouring": (_i, [_vp, _i, _vp, _vp]),
    "amg_eig_coarse_eigenvalues": (_i, [_vp, _vp]),
    "amg_eig_iterate": (_i, [_vp, _vp, _vp]),
    "amg_eig_destroy": (None, [_vp]),
    "amg_eig_strerror": (ctypes.c_char_p, [_i]),
    "amg_eig_last_error": (ctypes.c_char_p, [_vp]),
    "amg_eig_timing": (_i, [_vp, _i]),
    "amg_eig_site_stats": (_i, [_vp, _i, _vp, _vp, _vp]),
    "amg_eig_set_cpt": (_i, [_vp, _i, _i, _i]),
    "amg_eig_get_cpt": (_i, [_vp, _i, _i, _vp]),
    "amg_eig_tune_time": (_i, [_vp, _i, _i, _i, _i, _vp]),
    "amg_eig_galerkin": (_i, [_i64, _i64] + [_vp] * 14 + [_i64, _vp, _vp]),
    "amg_eig_strength": (_i, [_i64, _vp, _vp, _vp, _d, _vp, _vp]),
    "amg_eig_interpolation": (_i, [_i64] + [_vp] * 8 + [_i64, _vp, _vp, _vp]),
    "amg_eig_transpose": (_i, [_i64, _i64] + [_vp] * 6 + [_vp]),
    "amg_eig_pmis": (_i, [_i64] + [_vp] * 4 + [_i] + [_vp] * 3),
    "amg_eig_dense_sygv": (_i, [_i64] + [_vp] * 6),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class AmgEigError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__("%s (%d)%s" % (_lib.amg_eig_strerror(code).decode(), code, (": " + msg) if msg else ""))


def defaults(**kw):
    o = Opts()
    _lib.amg_eig_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _csr(rowptr, col, val, keep):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    keep.extend([rp, ci, va])
    return Csr(rp.size - 1, rp.ctypes.data, ci.ctypes.data, va.ctypes.data)


class Context:
    """One eigenproblem (A, M, q): host setup at construction, device work after bind()."""

    def __init__(self, rowptr, col, a, m, q, opts=None, m_rowptr=None, m_col=None):
        keep = []
        A = _csr(rowptr, col, a, keep)
        M = _csr(rowptr if m_rowptr is None else m_rowptr, col if m_col is None else m_col, m, keep)
        self._c = ctypes.c_void_p()
        self.opts = opts if opts is not None else defaults()
        rc = _lib.amg_eig_setup(ctypes.byref(A), ctypes.byref(M), int(q), ctypes.byref(self.opts),
                                ctypes.byref(self._c))
        if rc != OK:
            raise AmgEigError(rc)
        self.q = int(q)
        self.workspace = None
        self.stream = None
        self._static = False
        self._ws_bytes = 0

    # ----------------------------------------------------------- host side
    def _check(self, rc):
        if rc < 0:
            raise AmgEigError(rc, _lib.amg_eig_last_error(self._c).decode())
        return rc

    def footprint(self):
        n = ctypes.c_size_t()
        self._check(_lib.amg_eig_footprint(self._c, ctypes.byref(n)))
        return n.value

    def info(self):
        qe, nl = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.amg_eig_info(self._c, ctypes.byref(qe), ctypes.byref(nl), None))
        dims = np.zeros(nl.value, dtype=np.int64)
        self._check(_lib.amg_eig_info(self._c, None, None, _p(dims)))
        return {"qe": qe.value, "levels": nl.value, "dims": dims}

    def level_matrix(self, level):
        nnz = ctypes.c_int64()
        self._check(_lib.amg_eig_level_matrix(self._c, level, ctypes.byref(nnz), None, None, None, None))
        n = int(self.info()["dims"][level])
        rp = np.zeros(n + 1, np.int64)
        ci = np.zeros(nnz.value, np.int32)
        a = np.zeros(nnz.value)
        m = np.zeros(nnz.value)
        self._check(_lib.amg_eig_level_matrix(self._c, level, ctypes.byref(nnz), _p(rp), _p(ci), _p(a), _p(m)))
        return rp, ci, a, m

    def prolongation(self, level):
        nnz = ctypes.c_int64()
        self._check(_lib.amg_eig_level_prolongation(self._c, level, ctypes.byref(nnz), None, None, None))
        n = int(self.info()["dims"][level])
        rp = np.zeros(n + 1, np.int64)
        ci = np.zeros(nnz.value, np.int32)
        p = np.zeros(nnz.value)
        self._check(_lib.amg_eig_level_prolongation(self._c, level, ctypes.byref(nnz), _p(rp), _p(ci), _p(p)))
        return rp, ci, p

    def splitting(self, level):
        n = int(self.info()["dims"][level])
        cf = np.zeros(n, np.int32)
        self._check(_lib.amg_eig_level_splitting(self._c, level, _p(cf)))
        return cf

    def colouring(self, level):
        """Colours of level ``level``'s rows (multicolour Gauss-Seidel only)."""
        n = int(self.info()["dims"][level])
        colour = np.zeros(n, np.int32)
        nc = ctypes.c_int(0)
        self._check(_lib.amg_eig_level_colouring(self._c, level, _p(colour), ctypes.byref(nc)))
        return colour, nc.value

    def coarse_eigenvalues(self):
        lam = np.zeros(int(self.info()["dims"][-1]))
        self._check(_lib.amg_eig_coarse_eigenvalues(self._c, _p(lam)))
        return lam

    # --------------------------------------------------------- device side
    def bind(self, device="cuda", stream=None):
        import torch
        self.workspace = None  # a rebind releases the old workspace first
        self.workspace = torch.empty(self.footprint(), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        self._check(_lib.amg_eig_bind(self._c, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                      ctypes.c_void_p(self.stream.cuda_stream)))
        self._static, self._ws_bytes = False, self.workspace.numel()
        return self

    def bind_static(self, stream=None):
        """Bind to the library's static device workspace (no allocation; 64 MiB per
        device, one context at a time: binding another one unbinds this one).
        The current device and `stream` (default: its current stream)."""
        import torch
        self.workspace = None
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        size = ctypes.c_size_t()
        self._check(_lib.amg_eig_bind_static(self._c, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(size)))
        self._static, self._ws_bytes = True, size.value
        return self

    def init(self, mode=INIT_NESTED, seed=0, U=None):
        ptr, ldu = None, 0
        if U is not None:
            ptr, ldu = ctypes.c_void_p(U.data_ptr()), U.stride(0)
        self._check(_lib.amg_eig_init(self._c, mode, ctypes.c_uint64(seed), ptr, ldu))

    def correct(self, steps=1):
        self._check(_lib.amg_eig_correct(self._c, steps))

    def progress(self):
        """Ritz values, residuals, corrections done, convergence; "widened" is
        True when the block width control raised the width (the iterate is then
        discarded: bind again if `bound` is False, then init)."""
        qe = self.info()["qe"]
        th, rh = np.zeros(qe), np.zeros(qe)
        st, cv = ctypes.c_int(), ctypes.c_int()
        rc = self._check(_lib.amg_eig_progress(self._c, _p(th), _p(rh), ctypes.byref(st), ctypes.byref(cv)))
        widened = rc == WIDENED
        return {"theta": th, "rho": rh, "steps": st.value, "converged": bool(cv.value) and not widened,
                "widened": widened, "bound": not widened or self.footprint() <= self._ws_bytes}

    def solve(self, tol=1e-8, max_steps=100, U_out=None):
        """Algorithm 3.2 to max_{j<=q} rho_j <= tol; a widened block that needs a
        larger workspace is bound to a new one (same device and stream) and the
        solve starts again."""
        lam = np.zeros(self.q)
        ptr, ldu = None, 0
        if U_out is not None:
            ptr, ldu = ctypes.c_void_p(U_out.data_ptr()), U_out.stride(0)
        while True:
            rc = self._check(_lib.amg_eig_solve(self._c, tol, max_steps, _p(lam), ptr, ldu))
            if rc != WIDENED:
                return lam, rc == OK
            if self._static:
                self.bind_static(stream=self.stream)
            else:
                self.bind(device=self.workspace.device, stream=self.stream)

    def iterate(self):
        """The device iterate as a torch view (N x ld FP64, first qe columns used)
        into the caller's workspace (not available after bind_static: use
        solve(U_out=...) there)."""
        import torch
        if self._static:
            raise RuntimeError("no torch view of the static workspace; pass U_out to solve()")
        p = ctypes.c_void_p()
        ld = ctypes.c_int64()
        self._check(_lib.amg_eig_iterate(self._c, ctypes.byref(p), ctypes.byref(ld)))
        n = int(self.info()["dims"][0])
        off = p.value - self.workspace.data_ptr()
        return self.workspace[off:off + n * ld.value * 8].view(torch.float64).view(n, ld.value)

    def timing(self, enable=True):
        self._check(_lib.amg_eig_timing(self._c, 1 if enable else 0))

    def site_stats(self):
        """{site: (algorithmic bytes or flops per launch, total ms, launches)}."""
        out = {}
        for i, name in enumerate(SITES):
            b, ms, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
            self._check(_lib.amg_eig_site_stats(self._c, i, ctypes.byref(b), ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (b.value, ms.value, n.value)
        return out

    def level_nnz(self, level):
        nnz = ctypes.c_int64()
        self._check(_lib.amg_eig_level_matrix(self._c, level, ctypes.byref(nnz), None, None, None, None))
        return nnz.value

    def set_cpt(self, kind, level, cpt):
        """Columns per lane of the row kernels of one kind on one level (0: built-in rule)."""
        self._check(_lib.amg_eig_set_cpt(self._c, kind, level, cpt))

    def get_cpt(self, kind, level):
        v = ctypes.c_int()
        self._check(_lib.amg_eig_get_cpt(self._c, kind, level, ctypes.byref(v)))
        return v.value

    def tune_time(self, kind, level, cpt, reps=10):
        """Microseconds per pass of the row kernels of (kind, level) launched with cpt; clears the solve state."""
        us = ctypes.c_double()
        self._check(_lib.amg_eig_tune_time(self._c, kind, level, cpt, reps, ctypes.byref(us)))
        return us.value

    def close(self):
        if self._c:
            _lib.amg_eig_destroy(self._c)
            self._c = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def galerkin(n, nc, x_ptr, x_col, x_a, x_m, p_ptr, p_col, p_val, pt_ptr, pt_col, pt_val, stream=None):
    """Galerkin products P^T A P and P^T M P on the device (amg_eig_galerkin).

    All arguments are device tensors (int64 row pointers, int32 columns, float64
    values) on one device; returns device tensors (c_ptr, c_col, c_a, c_m).  A
    first call sizes the result, a second fills it."""
    dev = x_ptr.device
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    s = ctypes.c_void_p(stream.cuda_stream)
    ins = [x_ptr, x_col, x_a, x_m, p_ptr, p_col, p_val, pt_ptr, pt_col, pt_val]
    want = [torch.int64, torch.int32, torch.float64, torch.float64] + [torch.int64, torch.int32, torch.float64] * 2
    for t, d in zip(ins, want):
        if t.device != dev or t.dtype != d or not t.is_contiguous():
            raise ValueError("galerkin: arrays must be contiguous %s tensors on %s" % (d, dev))
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in ins]
    c_ptr = torch.empty(nc + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64()
    rc = _lib.amg_eig_galerkin(n, nc, *ptrs, ctypes.c_void_p(c_ptr.data_ptr()), None, None, None, 0,
                               ctypes.byref(nnz), s)
    if rc not in (OK, EWORKSPACE):
        raise AmgEigError(rc)
    cap = nnz.value
    c_col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    c_a = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    c_m = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    rc = _lib.amg_eig_galerkin(n, nc, *ptrs, ctypes.c_void_p(c_ptr.data_ptr()), ctypes.c_void_p(c_col.data_ptr()),
                               ctypes.c_void_p(c_a.data_ptr()), ctypes.c_void_p(c_m.data_ptr()), cap,
                               ctypes.byref(nnz), s)
    if rc != OK:
        raise AmgEigError(rc)
    return c_ptr, c_col[:cap], c_a[:cap], c_m[:cap]


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _stream_of(dev, stream):
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    return ctypes.c_void_p(stream.cuda_stream)


def strength(x_ptr, x_col, x_a, theta=0.25, stream=None):
    """Strong-coupling flags of eq. (2.1) on the device (amg_eig_strength): uint8 tensor per entry."""
    n = x_ptr.numel() - 1
    strong = torch.empty(max(x_col.numel(), 1), dtype=torch.uint8, device=x_ptr.device)
    rc = _lib.amg_eig_strength(n, _dptr(x_ptr), _dptr(x_col), _dptr(x_a), theta, _dptr(strong),
                               _stream_of(x_ptr.device, stream))
    if rc != OK:
        raise AmgEigError(rc)
    return strong[:x_col.numel()]


def pmis(x_ptr, x_col, strong, rnd, second_pass=False, stream=None):
    """PMIS C/F splitting on the device (amg_eig_pmis), optionally with the
    parallel second pass: (cf int32 device tensor, first-pass rounds)."""
    n = x_ptr.numel() - 1
    cf = torch.empty(max(n, 1), dtype=torch.int32, device=x_ptr.device)
    rounds = ctypes.c_int()
    rc = _lib.amg_eig_pmis(n, _dptr(x_ptr), _dptr(x_col), _dptr(strong), _dptr(rnd), int(bool(second_pass)), _dptr(cf),
                           ctypes.byref(rounds),
                           _stream_of(x_ptr.device, stream))
    if rc != OK:
        raise AmgEigError(rc)
    return cf[:n], rounds.value


def dense_sygv(A, M, stream=None):
    """A z = lambda M z on the device (amg_eig_dense_sygv) for n x n float64
    device tensors: (lam, Z, sweeps), Z^T M Z = I, eigenvalues ascending."""
    n = A.shape[0]
    dev = A.device
    for t in (A, M):
        if t.shape != (n, n) or t.dtype != torch.float64 or t.device != dev or not t.is_contiguous():
            raise ValueError("dense_sygv: A and M must be contiguous n x n float64 tensors on one device")
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Z = torch.empty((n, n), dtype=torch.float64, device=dev)
    sweeps = ctypes.c_int()
    rc = _lib.amg_eig_dense_sygv(n, _dptr(A), _dptr(M), _dptr(lam), _dptr(Z), ctypes.byref(sweeps),
                                 _stream_of(dev, stream))
    if rc != OK:
        raise AmgEigError(rc)
    return lam, Z, sweeps.value


def interpolation(x_ptr, x_col, x_a, strong, cf, stream=None):
    """Direct interpolation P of eqs. (2.2)-(2.4) on the device (amg_eig_interpolation).

    Returns device tensors (p_ptr, p_col, p_val) and the coarse size."""
    dev = x_ptr.device
    n = x_ptr.numel() - 1
    s = _stream_of(dev, stream)
    p_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nnz, nc = ctypes.c_int64(), ctypes.c_int64()
    args = [_dptr(x_ptr), _dptr(x_col), _dptr(x_a), _dptr(strong), _dptr(cf), _dptr(p_ptr)]
    rc = _lib.amg_eig_interpolation(n, *args, None, None, 0, ctypes.byref(nnz), ctypes.byref(nc), s)
    if rc not in (OK, EWORKSPACE):
        raise AmgEigError(rc)
    cap = nnz.value
    p_col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    p_val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    rc = _lib.amg_eig_interpolation(n, *args, _dptr(p_col), _dptr(p_val), cap, ctypes.byref(nnz),
                                    ctypes.byref(nc), s)
    if rc != OK:
        raise AmgEigError(rc)
    return p_ptr, p_col[:cap], p_val[:cap], nc.value


def transpose(p_ptr, p_col, p_val, nc, stream=None):
    """CSR transpose on the device (amg_eig_transpose): (pt_ptr, pt_col, pt_val)."""
    dev = p_ptr.device
    nr = p_ptr.numel() - 1
    nnz = p_col.numel()
    pt_ptr = torch.empty(nc + 1, dtype=torch.int64, device=dev)
    pt_col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    pt_val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    rc = _lib.amg_eig_transpose(nr, nc, _dptr(p_ptr), _dptr(p_col), _dptr(p_val), _dptr(pt_ptr), _dptr(pt_col),
                                _dptr(pt_val), _stream_of(dev, stream))
    if rc != OK:
        raise AmgEigError(rc)
    return pt_ptr, pt_col[:nnz], pt_val[:nnz]


def correct_batch(contexts, steps=1, stream=None):
    arr = (ctypes.c_void_p * len(contexts))(*[c._c.value for c in contexts])
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    rc = _lib.amg_eig_correct_batch(arr, len(contexts), steps, s)
    if rc < 0:
        raise AmgEigError(rc)


def _batch_error(rc, contexts):
    msgs = []
    for c in contexts:
        m = _lib.amg_eig_last_error(c._c)
        if m:
            msgs.append(m.decode())
    return AmgEigError(rc, "; ".join(dict.fromkeys(msgs)))


def correct_batch_joint(contexts, steps=1):
    """Correction steps for several requests with their small eigenproblems
    solved in shared launches (each member on its own bound stream)."""
    arr = (ctypes.c_void_p * max(1, len(contexts)))(*[c._c.value for c in contexts])
    rc = _lib.amg_eig_correct_batch_joint(arr, len(contexts), steps)
    if rc < 0:
        raise _batch_error(rc, contexts)


def init_batch_joint(contexts):
    """Nested start of several bound requests with the small eigenproblems of
    their coarse-level corrections solved in shared launches."""
    arr = (ctypes.c_void_p * max(1, len(contexts)))(*[c._c.value for c in contexts])
    rc = _lib.amg_eig_init_batch_joint(arr, len(contexts))
    if rc < 0:
        raise _batch_error(rc, contexts)


def from_problem(p, **opts):
    """Context for a workload dict (rowptr/col shared by A and M)."""
    return Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], defaults(**opts))
