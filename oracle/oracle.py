"""ctypes binding of the plain-C FP64 oracle (oracle.c).

TEST INFRASTRUCTURE: used by the tests, the smoke check and the benchmark's
CPU-baseline leg only. Every function mirrors one step of the method as the
C file describes it; this module only marshals numpy arrays.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

__all__ = [
    "build_oracle",
    "load",
    "Status",
    "spmv",
    "check",
    "edge_weights",
    "greedy_matching",
    "number_aggregates",
    "pairwise_prolongator",
    "restrict",
    "galerkin_pairwise",
    "l1_diag",
    "cholesky",
    "cholesky_solve",
    "smooth_w",
    "coarse_pcg",
    "smoothing_omega",
    "smooth_prolongator",
    "galerkin_general",
    "Hierarchy",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


class Status:
    OK = 0
    ERR_ARG = 1
    ERR_NOT_SYMMETRIC = 2
    ERR_NOT_SPD = 3
    ERR_STALL = 4
    ERR_OOM = 5
    ERR_BREAKDOWN = 7
    NOT_CONVERGED = 8


NATIVE_LIB_PATH = os.path.join(_HERE, "liboracle_native.so")


def build_oracle(force: bool = True, native: bool = False) -> str:
    """Compile liboracle.so with gcc (strict IEEE: no FP contraction).

    native=True compiles the copy used to time the oracle on a host,
    liboracle_native.so, with -O3 -march=native for that host's CPU. It keeps
    -ffp-contract=off and no fast-math, so no operation is fused or
    reassociated and its results are the same bits (a test checks this)."""
    path = NATIVE_LIB_PATH if native else _LIB_PATH
    if not force and os.path.exists(path):
        return path
    tmp = path + ".tmp%d" % os.getpid()
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", *opt, "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, path)
    return path


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rp", C.POINTER(C.c_int32)),
                ("ci", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


_lib = None
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def load():
    """Loads liboracle.so (building it if absent). ORACLE_LIB names another
    build of oracle.c to load instead (the mutation tests use it to check
    that the pins reject a planted mistake)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB") or _LIB_PATH
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build_oracle()
    lib = C.CDLL(path)
    P = C.POINTER(_Csr)
    sig = {
        "orc_spmv": (None, [P, _F64P, _F64P]),
        "orc_check": (C.c_int, [P]),
        "orc_num_edges": (C.c_int64, [P]),
        "orc_edge_weights": (None, [P, _F64P, _I32P, _I32P, _F64P]),
        "orc_greedy_matching": (C.c_int64, [C.c_int32, C.c_int64, _I32P, _I32P, _F64P, _I32P]),
        "orc_number_aggregates": (C.c_int32, [C.c_int32, _I32P, _I32P]),
        "orc_pairwise_prolongator": (None, [C.c_int32, _I32P, _F64P, _F64P]),
        "orc_restrict": (None, [C.c_int32, C.c_int32, _I32P, _F64P, _F64P, _F64P]),
        "orc_galerkin_pairwise": (C.c_int, [P, C.c_int32, _I32P, _F64P, P]),
        "orc_csr_free": (None, [P]),
        "orc_l1_diag": (None, [P, _F64P]),
        "orc_cholesky": (C.c_int, [C.c_int32, _F64P]),
        "orc_cholesky_solve": (None, [C.c_int32, _F64P, _F64P, _F64P]),
        "orc_coarse_pcg": (C.c_int32, [P, _F64P, _F64P, C.c_double, C.c_int32, _F64P]),
        "orc_smoothing_omega": (C.c_double, [P]),
        "orc_smooth_prolongator": (C.c_int, [P, C.c_int32, _I32P, _F64P, C.c_double, P]),
        "orc_galerkin_general": (C.c_int, [P, P, C.c_int32, P]),
        "orc_setup_opts": (C.c_int, [P, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_void_p)]),
        "orc_level_pbar_nnz": (C.c_int64, [C.c_void_p, C.c_int32]),
        "orc_level_pbar": (None, [C.c_void_p, C.c_int32, _I32P, _I32P, _F64P]),
        "orc_level_omega": (C.c_double, [C.c_void_p, C.c_int32]),
        "orc_set_coarse_solver": (None, [C.c_void_p, C.c_int32, C.c_double, C.c_int32]),
        "orc_setup": (C.c_int, [P, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                C.POINTER(C.c_void_p)]),
        "orc_free": (None, [C.c_void_p]),
        "orc_num_levels": (C.c_int32, [C.c_void_p]),
        "orc_level_n": (C.c_int64, [C.c_void_p, C.c_int32]),
        "orc_level_nnz": (C.c_int64, [C.c_void_p, C.c_int32]),
        "orc_level_csr": (None, [C.c_void_p, C.c_int32, _I32P, _I32P, _F64P]),
        "orc_level_transfer": (None, [C.c_void_p, C.c_int32, _I32P, _F64P]),
        "orc_level_l1diag": (None, [C.c_void_p, C.c_int32, _F64P]),
        "orc_level_w": (None, [C.c_void_p, C.c_int32, _F64P]),
        "orc_level_sweeps": (C.c_int32, [C.c_void_p, C.c_int32]),
        "orc_coarse_factor": (None, [C.c_void_p, _F64P]),
        "orc_vcycle": (None, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _F64P, _F64P]),
        "orc_smooth_w": (None, [P, C.c_int32, _F64P]),
        "orc_kcycle": (None, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _F64P, _F64P]),
        "orc_fcg2": (None, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _F64P, _F64P]),
        "orc_fcg": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _F64P, _F64P,
                              C.c_double, C.c_int32, _F64P]),
        "orc_pcg": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _F64P, _F64P, C.c_double,
                              C.c_int32, _F64P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class _HostCsr:
    """Keeps numpy arrays alive behind a ctypes CSR struct."""

    def __init__(self, A):
        self.rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        self.ci = np.ascontiguousarray(A.col, dtype=np.int32)
        self.val = np.ascontiguousarray(A.val, dtype=np.float64)
        self.s = _Csr(int(A.n), int(self.ci.shape[0]),
                      self.rp.ctypes.data_as(C.POINTER(C.c_int32)),
                      self.ci.ctypes.data_as(C.POINTER(C.c_int32)),
                      self.val.ctypes.data_as(C.POINTER(C.c_double)))

    @property
    def ref(self):
        return C.byref(self.s)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def spmv(A, x):
    lib = load()
    h = _HostCsr(A)
    y = np.empty(A.n)
    lib.orc_spmv(h.ref, _f64(x), y)
    return y


def check(A) -> int:
    return load().orc_check(_HostCsr(A).ref)


def edge_weights(A, w=None):
    """Returns (lo, hi, c) for every undirected edge (eq. (weights))."""
    lib = load()
    h = _HostCsr(A)
    ne = lib.orc_num_edges(h.ref)
    lo = np.empty(ne, dtype=np.int32)
    hi = np.empty(ne, dtype=np.int32)
    c = np.empty(ne)
    w = np.ones(A.n) if w is None else _f64(w)
    lib.orc_edge_weights(h.ref, w, lo, hi, c)
    return lo, hi, c


def greedy_matching(n, lo, hi, c):
    mate = np.empty(n, dtype=np.int32)
    nm = load().orc_greedy_matching(n, len(lo), _i32(lo), _i32(hi), _f64(c), mate)
    return mate, int(nm)


def number_aggregates(mate):
    n = len(mate)
    agg = np.empty(n, dtype=np.int32)
    nc = load().orc_number_aggregates(n, _i32(mate), agg)
    return agg, int(nc)


def pairwise_prolongator(mate, w):
    n = len(mate)
    p = np.empty(n)
    load().orc_pairwise_prolongator(n, _i32(mate), _f64(w), p)
    return p


def restrict(agg, p, v, nc):
    vc = np.empty(nc)
    load().orc_restrict(len(agg), nc, _i32(agg), _f64(p), _f64(v), vc)
    return vc


def galerkin_pairwise(A, agg, p, nc):
    from paper_2006_16147_amd.inputs import Csr

    lib = load()
    h = _HostCsr(A)
    out = _Csr()
    st = lib.orc_galerkin_pairwise(h.ref, nc, _i32(agg), _f64(p), C.byref(out))
    if st:
        raise RuntimeError("orc_galerkin_pairwise failed: %d" % st)
    nnz = int(out.nnz)
    rp = np.ctypeslib.as_array(out.rp, shape=(nc + 1,)).copy()
    ci = np.ctypeslib.as_array(out.ci, shape=(max(nnz, 1),))[:nnz].copy()
    val = np.ctypeslib.as_array(out.val, shape=(max(nnz, 1),))[:nnz].copy()
    lib.orc_csr_free(C.byref(out))
    return Csr(nc, rp, ci, val)


def l1_diag(A):
    m = np.empty(A.n)
    load().orc_l1_diag(_HostCsr(A).ref, m)
    return m


def cholesky(a):
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    st = load().orc_cholesky(a.shape[0], a)
    return st, a


def cholesky_solve(L, r):
    L = _f64(L)
    z = np.empty(L.shape[0])
    load().orc_cholesky_solve(L.shape[0], L, _f64(r), z)
    return z


def coarse_pcg(A, m, b, rtol=1e-4, maxit=30):
    """CG from zero preconditioned by the diagonal m, stopped on the first
    ||r_k|| < rtol ||b|| or after maxit iterations (Section 5's coarsest
    solver). Returns (x, iterations)."""
    x = np.empty(A.n)
    it = load().orc_coarse_pcg(_HostCsr(A).ref, _f64(m), _f64(b), float(rtol), int(maxit), x)
    return x, int(it)


def _take_csr(out, nrows):
    """Copies a C-allocated CSR into numpy (rp, ci, val) and frees it."""
    nnz = int(out.nnz)
    rp = np.ctypeslib.as_array(out.rp, shape=(nrows + 1,)).copy()
    ci = np.ctypeslib.as_array(out.ci, shape=(max(nnz, 1),))[:nnz].copy()
    val = np.ctypeslib.as_array(out.val, shape=(max(nnz, 1),))[:nnz].copy()
    load().orc_csr_free(C.byref(out))
    return rp, ci, val


class _RectCsr:
    """A rows x cols CSR given as (rp, ci, val) (the struct holds rows only)."""

    def __init__(self, rp, ci, val):
        self.n = len(rp) - 1
        self.row_ptr, self.col, self.val = rp, ci, val


def smoothing_omega(A):
    """1 / ||D^-1 A||_inf."""
    return float(load().orc_smoothing_omega(_HostCsr(A).ref))


def smooth_prolongator(A, nc, agg, p, omega):
    """Pbar = (I - omega D^-1 A) P as (rp, ci, val), n x nc."""
    out = _Csr()
    st = load().orc_smooth_prolongator(_HostCsr(A).ref, int(nc), _i32(agg), _f64(p),
                                       float(omega), C.byref(out))
    if st:
        raise RuntimeError("orc_smooth_prolongator failed: %d" % st)
    return _take_csr(out, A.n)


def galerkin_general(A, Pb, nc):
    """Pbar^T A Pbar for Pbar = (rp, ci, val) with nc columns; returns a Csr."""
    from paper_2006_16147_amd.inputs import Csr

    out = _Csr()
    st = load().orc_galerkin_general(_HostCsr(A).ref, _HostCsr(_RectCsr(*Pb)).ref, int(nc),
                                     C.byref(out))
    if st:
        raise RuntimeError("orc_galerkin_general failed: %d" % st)
    return Csr(int(nc), *_take_csr(out, int(nc)))


def smooth_w(A, nu, w0=None):
    """nu l1-Jacobi iterations on A w = 0 from the sample w0 (ones if None)."""
    lib = load()
    w = np.ones(A.n) if w0 is None else np.array(w0, dtype=np.float64, copy=True)
    hc = _HostCsr(A)
    lib.orc_smooth_w(hc.ref, int(nu), w)
    return w


class Hierarchy:
    """Oracle multilevel hierarchy (Sections 3.1-3.3)."""

    def __init__(self, A, w=None, sweeps=3, max_coarse=200, max_levels=32, coarse=None,
                 smooth=False):
        """coarse: None for the dense Cholesky coarsest solve, or (rtol, maxit)
        for the iterative one (CG with the l1-Jacobi diagonal). smooth: build
        the levels with the smoothed prolongators."""
        lib = load()
        self._lib = lib
        self._h = C.c_void_p()
        hc = _HostCsr(A)
        wv = None
        if w is not None:
            self._w = _f64(w)
            wv = self._w.ctypes.data_as(C.c_void_p)
        self.status = lib.orc_setup_opts(hc.ref, wv, sweeps, max_coarse, max_levels,
                                         1 if smooth else 0, C.byref(self._h))
        if self.status != Status.OK:
            self._h = None
        elif coarse is not None:
            lib.orc_set_coarse_solver(self._h, 1, float(coarse[0]), int(coarse[1]))

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_free(self._h)
            self._h = None

    @property
    def ok(self):
        return self._h is not None

    @property
    def num_levels(self) -> int:
        return int(self._lib.orc_num_levels(self._h))

    def level_n(self, l):
        return int(self._lib.orc_level_n(self._h, l))

    def level_nnz(self, l):
        return int(self._lib.orc_level_nnz(self._h, l))

    def sizes(self):
        return [self.level_n(l) for l in range(self.num_levels)]

    def nnzs(self):
        return [self.level_nnz(l) for l in range(self.num_levels)]

    def level_csr(self, l):
        from paper_2006_16147_amd.inputs import Csr

        n, nnz = self.level_n(l), self.level_nnz(l)
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz)
        self._lib.orc_level_csr(self._h, l, rp, ci, val)
        return Csr(n, rp, ci, val)

    def transfer(self, l):
        n = self.level_n(l)
        agg = np.empty(n, dtype=np.int32)
        p = np.empty(n)
        self._lib.orc_level_transfer(self._h, l, agg, p)
        return agg, p

    def l1diag(self, l):
        m = np.empty(self.level_n(l))
        self._lib.orc_level_l1diag(self._h, l, m)
        return m

    def w(self, l):
        w = np.empty(self.level_n(l))
        self._lib.orc_level_w(self._h, l, w)
        return w

    def sweeps_run(self, l):
        return int(self._lib.orc_level_sweeps(self._h, l))

    def pbar(self, l):
        """Smoothed prolongator of level l as (rp, ci, val), n_l x n_{l+1}."""
        n, nnz = self.level_n(l), int(self._lib.orc_level_pbar_nnz(self._h, l))
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(max(nnz, 1), dtype=np.int32)
        val = np.empty(max(nnz, 1))
        self._lib.orc_level_pbar(self._h, l, rp, ci, val)
        return rp, ci[:nnz], val[:nnz]

    def omega(self, l):
        return float(self._lib.orc_level_omega(self._h, l))

    def coarse_factor(self):
        nL = self.level_n(self.num_levels - 1)
        L = np.empty((nL, nL))
        self._lib.orc_coarse_factor(self._h, L)
        return L

    def opc(self):
        z = self.nnzs()
        return sum(z) / z[0]

    def vcycle(self, r, l=0, pre=1, post=1):
        z = np.empty(self.level_n(l))
        self._lib.orc_vcycle(self._h, l, pre, post, _f64(r), z)
        return z

    def kcycle(self, r, l=0, pre=1, post=1):
        """K-cycle on level l (Section 3.1)."""
        z = np.empty(self.level_n(l))
        self._lib.orc_kcycle(self._h, l, pre, post, _f64(r), z)
        return z

    def fcg2(self, b, m, pre=1, post=1):
        """The K-cycle's two flexible-CG iterations on level m, from zero."""
        x = np.empty(self.level_n(m))
        self._lib.orc_fcg2(self._h, m, pre, post, _f64(b), x)
        return x

    def fcg(self, b, x0=None, rtol=1e-6, maxit=500, pre=1, post=1, cycle="K"):
        """Flexible CG with the K-cycle (cycle="K") or V-cycle ("V")."""
        n = self.level_n(0)
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        out = np.zeros(4)
        st = self._lib.orc_fcg(self._h, 1 if cycle == "K" else 0, pre, post, _f64(b), x, rtol,
                               maxit, out)
        return x, {"status": int(st), "iterations": int(out[0]), "converged": bool(out[1]),
                   "rel_res": float(out[2]), "rel_res_true": float(out[3])}

    def pcg(self, b, x0=None, rtol=1e-6, maxit=500, pre=1, post=1):
        n = self.level_n(0)
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        out = np.zeros(4)
        st = self._lib.orc_pcg(self._h, pre, post, _f64(b), x, rtol, maxit, out)
        return x, {"status": int(st), "iterations": int(out[0]), "converged": bool(out[1]),
                   "rel_res": float(out[2]), "rel_res_true": float(out[3])}
