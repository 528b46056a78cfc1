"""Thin ctypes binding of the HIP C ABI (include/amg.h).

Functions carry the ABI's names and only marshal arguments: torch tensors on
the current HIP device are passed by ``data_ptr()``, results are copied into
numpy arrays. Every numerical step runs in the HIP library; if the library
is not built this module raises instead of computing anything itself.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "AmgError", "Status", "FP64", "FP32", "FLAG_NO_GRAPH", "FLAG_SKIP_CHECKS", "MAX_DENSE",
    "lib_path", "load_library", "Params", "SolveInfo", "Hierarchy",
    "amg_params_default", "amg_setup", "amg_pcg_solve", "amg_pcg_solve_batch",
    "amg_vcycle_apply", "amg_free", "amg_estimate_footprint", "amg_status_string",
    "amg_wait", "amg_query", "amg_pcg_solve_noalloc", "FLAG_ASYNC", "EXPORTED_SYMBOLS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
FP64, FP32 = 0, 1
CYCLE_V, CYCLE_K = 0, 1
COARSE_CHOLESKY, COARSE_PCG = 0, 1
FLAG_NO_GRAPH, FLAG_SKIP_CHECKS, FLAG_NO_VALUE_COMPRESSION, FLAG_ASYNC = 1, 2, 4, 8
TIME_IN_SOLVE = 16  # amg_time_kernel: time the kernel inside the CG iterations
MAX_DENSE = 4096

EXPORTED_SYMBOLS = (
    "amg_params_default", "amg_setup", "amg_pcg_solve", "amg_pcg_solve_batch",
    "amg_vcycle_apply", "amg_set_stream", "amg_free", "amg_num_levels", "amg_level_info", "amg_get_level_csr",
    "amg_get_transfer", "amg_get_l1diag", "amg_get_w", "amg_footprint_bytes",
    "amg_estimate_footprint", "amg_setup_times", "amg_matching_rounds", "amg_time_kernel",
    "amg_batch_tile", "amg_status_string", "amg_get_prolongator", "amg_get_aggregates",
    "amg_wait", "amg_query", "amg_pcg_solve_noalloc",
)


class Status:
    OK = 0
    ERR_ARG = 1
    ERR_NOT_SYMMETRIC = 2
    ERR_NOT_SPD = 3
    ERR_STALL = 4
    ERR_OOM = 5
    ERR_HIP = 6
    ERR_BREAKDOWN = 7
    NOT_CONVERGED = 8


class AmgError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = int(status)
        msg = load_library().amg_status_string(self.status).decode()
        super().__init__("%s: %s (status %d)" % (where, msg, self.status))


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("max_coarse", C.c_int32), ("max_levels", C.c_int32),
                ("pre", C.c_int32), ("post", C.c_int32), ("precision", C.c_int32),
                ("w", C.c_void_p), ("stream", C.c_void_p), ("device", C.c_int32),
                ("flags", C.c_int32),
                ("cycle", C.c_int32), ("w_sweeps", C.c_int32), ("coarse_solver", C.c_int32),
                ("coarse_maxit", C.c_int32), ("coarse_rtol", C.c_double),
                ("smooth_p", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double), ("converged", C.c_int32), ("ms", C.c_double)]

    def as_dict(self):
        return {"iterations": int(self.iterations), "converged": bool(self.converged),
                "rel_res_recursive": float(self.rel_res_recursive),
                "rel_res_true": float(self.rel_res_true), "ms": float(self.ms)}


_lib = None


def lib_path() -> str:
    return os.path.join(_HERE, "libamg_hip.so")


def load_library():
    """Loads libamg_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is missing: run `python -c \"import __graft_entry__ as "
                           "g; g.build()\"` (or paper_2006_16147_amd/build.py) first" % path)
    L = C.CDLL(path)
    P, V, I32, I64, D = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "amg_params_default": (None, [P(Params)]),
        "amg_setup": (C.c_int, [P(Csr), P(Params), P(V)]),
        "amg_pcg_solve": (C.c_int, [V, V, V, D, I32, P(SolveInfo)]),
        "amg_pcg_solve_batch": (C.c_int, [V, I32, V, V, D, I32, P(SolveInfo)]),
        "amg_pcg_solve_noalloc": (C.c_int, [V, V, V, D, I32, P(SolveInfo)]),
        "amg_vcycle_apply": (C.c_int, [V, V, V]),
        "amg_set_stream": (C.c_int, [V, V]),
        "amg_wait": (C.c_int, [V]),
        "amg_query": (C.c_int, [V, P(I32)]),
        "amg_get_aggregates": (C.c_int, [V, I32, V]),
        "amg_free": (None, [V]),
        "amg_num_levels": (C.c_int, [V, P(I32)]),
        "amg_level_info": (C.c_int, [V, I32, P(I64), P(I64)]),
        "amg_get_level_csr": (C.c_int, [V, I32, V, V, V]),
        "amg_get_transfer": (C.c_int, [V, I32, V, V]),
        "amg_get_l1diag": (C.c_int, [V, I32, V]),
        "amg_get_prolongator": (C.c_int, [V, I32, P(I64), V, V, V, P(D)]),
        "amg_get_w": (C.c_int, [V, I32, V]),
        "amg_footprint_bytes": (C.c_size_t, [V]),
        "amg_estimate_footprint": (C.c_size_t, [I64, I64, P(Params)]),
        "amg_setup_times": (C.c_int, [V, V]),
        "amg_matching_rounds": (C.c_int, [V, I32, P(I32)]),
        "amg_time_kernel": (C.c_int, [V, I32, I32, I32, P(D), P(D)]),
        "amg_batch_tile": (C.c_int, [V, P(I32), P(I32)]),
        "amg_status_string": (C.c_char_p, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(t, dtype=None, what="array"):
    """Device pointer of a contiguous torch tensor on the GPU."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor on the GPU" % what)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % what)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return t.data_ptr()


def amg_params_default(**overrides) -> Params:
    p = Params()
    load_library().amg_params_default(C.byref(p))
    for k, v in overrides.items():
        if k == "stream":
            v = v.cuda_stream if hasattr(v, "cuda_stream") else v
        if k == "w" and v is not None and not isinstance(v, int):
            import torch

            v = _ptr(v, torch.float64, "w")
        setattr(p, k, v if v is not None else None)
    return p


def amg_status_string(status: int) -> str:
    return load_library().amg_status_string(int(status)).decode()


def amg_estimate_footprint(n: int, nnz: int, params: Params | None = None) -> int:
    p = params if params is not None else amg_params_default()
    return int(load_library().amg_estimate_footprint(int(n), int(nnz), C.byref(p)))


class Hierarchy:
    """Owner of an amg_hierarchy handle (amg_free on close/deletion)."""

    def __init__(self, handle, n, device=0, is_async=False):
        self._h = C.c_void_p(handle)
        self.n = int(n)
        self.device = int(device)
        self.is_async = bool(is_async)
        self._pending = None  # (info, keep-alive references) of an AMG_ASYNC solve

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().amg_free(self._h)  # waits for a solve in flight
            self._h = C.c_void_p(0)
            self._pending = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, where):
        if st != Status.OK:
            raise AmgError(st, where)

    @property
    def num_levels(self) -> int:
        v = C.c_int32()
        self._check(load_library().amg_num_levels(self._h, C.byref(v)), "amg_num_levels")
        return int(v.value)

    def level_info(self, l):
        n, nnz = C.c_int64(), C.c_int64()
        self._check(load_library().amg_level_info(self._h, l, C.byref(n), C.byref(nnz)),
                    "amg_level_info")
        return int(n.value), int(nnz.value)

    def sizes(self):
        return [self.level_info(l)[0] for l in range(self.num_levels)]

    def nnzs(self):
        return [self.level_info(l)[1] for l in range(self.num_levels)]

    def opc(self):
        z = self.nnzs()
        return sum(z) / z[0]

    def level_csr(self, l):
        n, nnz = self.level_info(l)
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz, dtype=np.float64)
        self._check(load_library().amg_get_level_csr(self._h, l, rp.ctypes.data,
                                                     ci.ctypes.data, val.ctypes.data),
                    "amg_get_level_csr")
        return rp, ci, val

    def aggregates(self, l):
        n, _ = self.level_info(l)
        agg = np.empty(n, dtype=np.int32)
        self._check(load_library().amg_get_aggregates(self._h, l, agg.ctypes.data),
                    "amg_get_aggregates")
        return agg

    def transfer(self, l):
        n, _ = self.level_info(l)
        agg = np.empty(n, dtype=np.int32)
        p = np.empty(n, dtype=np.float64)
        self._check(load_library().amg_get_transfer(self._h, l, agg.ctypes.data, p.ctypes.data),
                    "amg_get_transfer")
        return agg, p

    def prolongator(self, l):
        """Smoothed prolongator of level l: ((rp, ci, val), omega)."""
        L = load_library()
        nnz, om = C.c_int64(), C.c_double()
        self._check(L.amg_get_prolongator(self._h, l, C.byref(nnz), None, None, None, None),
                    "amg_get_prolongator")
        n, _ = self.level_info(l)
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(max(nnz.value, 1), dtype=np.int32)
        val = np.empty(max(nnz.value, 1))
        self._check(L.amg_get_prolongator(self._h, l, C.byref(nnz), rp.ctypes.data,
                                          ci.ctypes.data, val.ctypes.data, C.byref(om)),
                    "amg_get_prolongator")
        return (rp, ci[:nnz.value], val[:nnz.value]), om.value

    def l1diag(self, l):
        n, _ = self.level_info(l)
        m = np.empty(n)
        self._check(load_library().amg_get_l1diag(self._h, l, m.ctypes.data), "amg_get_l1diag")
        return m

    def w(self, l):
        n, _ = self.level_info(l)
        w = np.empty(n)
        self._check(load_library().amg_get_w(self._h, l, w.ctypes.data), "amg_get_w")
        return w

    def set_stream(self, stream):
        """Orders later calls after `stream` (a torch stream or a raw handle)."""
        raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        self._check(load_library().amg_set_stream(self._h, raw), "amg_set_stream")

    def footprint_bytes(self) -> int:
        return int(load_library().amg_footprint_bytes(self._h))

    def setup_times(self):
        ms = np.zeros(8)
        self._check(load_library().amg_setup_times(self._h, ms.ctypes.data), "amg_setup_times")
        keys = ["validate", "matching", "numbering", "galerkin", "compose", "smoother_coarsest",
                "solve_format", "total"]
        return dict(zip(keys, ms.tolist()))

    def matching_rounds(self, l):
        v = C.c_int32()
        self._check(load_library().amg_matching_rounds(self._h, l, C.byref(v)),
                    "amg_matching_rounds")
        return int(v.value)

    def batch_tile(self) -> int:
        return self.batch_tiles()[0]

    def batch_tiles(self):
        """(one-value column tile, vector tile shift) chosen by the autotuner."""
        v, sh = C.c_int32(), C.c_int32()
        self._check(load_library().amg_batch_tile(self._h, C.byref(v), C.byref(sh)),
                    "amg_batch_tile")
        return int(v.value), int(sh.value)

    def time_kernel(self, kernel, level=0, reps=20):
        ms, by = C.c_double(), C.c_double()
        self._check(load_library().amg_time_kernel(self._h, kernel, level, reps, C.byref(ms),
                                                   C.byref(by)), "amg_time_kernel")
        return float(ms.value), float(by.value)


def amg_setup(row_ptr, col, val, params: Params | None = None, **kw) -> Hierarchy:
    """Builds the hierarchy of a CSR matrix given as torch GPU tensors."""
    import torch

    n = row_ptr.numel() - 1
    A = Csr(n, col.numel(), _ptr(row_ptr, torch.int32, "row_ptr"), _ptr(col, torch.int32, "col"),
            _ptr(val, torch.float64, "val"))
    if params is None and "stream" not in kw:
        kw["stream"] = torch.cuda.current_stream().cuda_stream
    p = params if params is not None else amg_params_default(**kw)
    out = C.c_void_p()
    st = load_library().amg_setup(C.byref(A), C.byref(p), C.byref(out))
    if st != Status.OK:
        raise AmgError(st, "amg_setup")
    device = p.device if p.device >= 0 else torch.cuda.current_device()
    return Hierarchy(out.value, n, device, bool(p.flags & FLAG_ASYNC))


def _check_vectors(h: Hierarchy, shape, **tensors):
    """Rejects, before any launch, tensors whose shape or device does not
    match the hierarchy (the library would read or write past them)."""
    for name, t in tensors.items():
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s has shape %s, the hierarchy needs %s"
                             % (name, tuple(t.shape), tuple(shape)))
        if t.is_cuda and t.device.index != h.device:
            raise ValueError("%s is on cuda:%s, the hierarchy on cuda:%d"
                             % (name, t.device.index, h.device))


def amg_pcg_solve(h: Hierarchy, b, x, rtol=1e-8, maxit=1000, raise_on_error=True):
    """Solves into x (torch float64 on the GPU, in: x0); returns (status, info)."""
    import torch

    _check_vectors(h, (h.n,), b=b, x=x)
    info = SolveInfo()
    st = load_library().amg_pcg_solve(h.handle, _ptr(b, torch.float64, "b"),
                                      _ptr(x, torch.float64, "x"), float(rtol), int(maxit),
                                      C.byref(info))
    if h.is_async and st == Status.OK:
        h._pending = (lambda: info.as_dict(), (info, b, x))
        return st, None  # amg_wait(h) gives the status and info
    if raise_on_error and st not in (Status.OK, Status.NOT_CONVERGED):
        raise AmgError(st, "amg_pcg_solve")
    return st, info.as_dict()


def amg_pcg_solve_noalloc(h: Hierarchy, b, x, rtol=1e-8, maxit=1000, raise_on_error=True):
    """amg_pcg_solve without any device allocation in the call (its scratch
    is the library's static device array); always blocking."""
    import torch

    _check_vectors(h, (h.n,), b=b, x=x)
    info = SolveInfo()
    st = load_library().amg_pcg_solve_noalloc(h.handle, _ptr(b, torch.float64, "b"),
                                              _ptr(x, torch.float64, "x"), float(rtol),
                                              int(maxit), C.byref(info))
    if raise_on_error and st not in (Status.OK, Status.NOT_CONVERGED):
        raise AmgError(st, "amg_pcg_solve_noalloc")
    return st, info.as_dict()


def amg_pcg_solve_batch(h: Hierarchy, B, X, rtol=1e-8, maxit=1000, raise_on_error=True):
    """Solves the k columns of the n x k row-major blocks B, X; returns (status, [info])."""
    import torch

    if B.dim() != 2:
        raise ValueError("B must be a 2-D n x k tensor, got shape %s" % (tuple(B.shape),))
    k = B.shape[1]
    _check_vectors(h, (h.n, k), B=B, X=X)
    infos = (SolveInfo * max(k, 1))()
    st = load_library().amg_pcg_solve_batch(h.handle, k, _ptr(B, torch.float64, "B"),
                                            _ptr(X, torch.float64, "X"), float(rtol), int(maxit),
                                            infos)
    if h.is_async and st == Status.OK and k > 0:
        h._pending = (lambda: [infos[j].as_dict() for j in range(k)], (infos, B, X))
        return st, None  # amg_wait(h) gives the status and the infos
    if raise_on_error and st not in (Status.OK, Status.NOT_CONVERGED):
        raise AmgError(st, "amg_pcg_solve_batch")
    return st, [infos[j].as_dict() for j in range(k)]


def amg_wait(h: Hierarchy, raise_on_error=True):
    """Waits for the AMG_ASYNC solve in flight on h; returns (status, info)
    as the blocking call would have (info None when nothing was in flight)."""
    st = load_library().amg_wait(h.handle)
    pending, h._pending = h._pending, None
    if raise_on_error and st not in (Status.OK, Status.NOT_CONVERGED):
        raise AmgError(st, "amg_wait")
    return st, (pending[0]() if pending else None)


def amg_query(h: Hierarchy) -> bool:
    """True when no AMG_ASYNC solve is in flight on h or it has finished."""
    done = C.c_int32()
    st = load_library().amg_query(h.handle, C.byref(done))
    if st != Status.OK:
        raise AmgError(st, "amg_query")
    return bool(done.value)


def amg_vcycle_apply(h: Hierarchy, r, z):
    import torch

    _check_vectors(h, (h.n,), r=r, z=z)
    st = load_library().amg_vcycle_apply(h.handle, _ptr(r, torch.float64, "r"),
                                         _ptr(z, torch.float64, "z"))
    if st != Status.OK:
        raise AmgError(st, "amg_vcycle_apply")


def amg_free(h: Hierarchy):
    h.close()
