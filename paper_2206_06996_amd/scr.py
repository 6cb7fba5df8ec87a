"""ctypes binding of libscr.so with the names of include/scr.h.

Argument marshalling only: every computation runs in the HIP library.  Device buffers are torch
CUDA tensors (ROCm); the stream is torch's current stream unless one is passed.  There is no CPU
fallback: a missing library or device raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscr.so")
_lib = None
P = C.c_void_p

SCR_OK, SCR_NOT_CONVERGED = 0, 1
SCR_E_INVALID, SCR_E_OOM, SCR_E_HIP, SCR_E_BREAKDOWN, SCR_E_UNIMPLEMENTED, SCR_E_NO_DEVICE = -1, -2, -3, -4, -5, -6
SCR_SYSTEM, MESH_SYSTEM = 0, 1
SCR_FP64, SCR_MIXED = 0, 1
SCR_SMOOTH_JACOBI, SCR_SMOOTH_CHEBYSHEV = 0, 1

EXPORTED = ["scr_default_amg_opts", "scr_default_solve_opts", "scr_ctx_create", "scr_ctx_destroy",
            "scr_ctx_bytes_in_use", "amg_setup", "scr_solve", "mesh_motion_solve", "scr_handle_destroy",
            "scr_handle_bytes", "scr_footprint_estimate", "scr_status_str", "scr_last_error", "scr_hier_levels",
            "scr_hier_level_info", "scr_hier_level_copy", "scr_matrix_copy", "scr_apply", "scr_ctx_profile",
            "scr_ctx_profile_read"]
SCR_PROF_OFF, SCR_PROF_SMOOTH_A0 = 0, 1


class ScrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class ScrBsr(C.Structure):
    _fields_ = [("n_brows", C.c_int32), ("bs", C.c_int32), ("nnzb", C.c_int64), ("row_ptr", P),
                ("col_idx", P), ("val", P)]


class AmgOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("theta", C.c_double), ("smoother", C.c_int), ("cheb_degree", C.c_int),
                ("cheb_ratio", C.c_double), ("jacobi_sweeps", C.c_int), ("coarse_max", C.c_int),
                ("max_levels", C.c_int), ("max_coarse_ratio", C.c_double), ("seed", C.c_uint64)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_A", C.c_double), ("tol_S", C.c_double), ("tol_I", C.c_double),
                ("max_it", C.c_int), ("max_it_A", C.c_int), ("max_it_S", C.c_int), ("max_it_I", C.c_int),
                ("restart", C.c_int), ("restart_inner", C.c_int), ("use_x0", C.c_int), ("flexible_cg", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("outer_it", C.c_int), ("converged", C.c_int), ("rel_res_true", C.c_double),
                ("calls_A", C.c_int64), ("its_A", C.c_int64), ("calls_S", C.c_int64), ("its_S", C.c_int64),
                ("calls_I", C.c_int64), ("its_I", C.c_int64), ("vcycles_A", C.c_int64), ("vcycles_S", C.c_int64),
                ("vcycles_L", C.c_int64), ("mesh_its", C.c_int64 * 3), ("mesh_rel", C.c_double * 3),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double), ("device_bytes", C.c_int64)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if not isinstance(v, (int, float)) else v
        return d


def lib():
    """Load libscr.so (built by paper_2206_06996_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.scr_default_amg_opts.argtypes = [C.POINTER(AmgOpts)]
        L.scr_default_solve_opts.argtypes = [C.POINTER(SolveOpts)]
        L.scr_ctx_create.argtypes = [C.c_int, C.c_int64, C.POINTER(P)]
        L.scr_ctx_destroy.argtypes = [P]
        L.scr_ctx_bytes_in_use.argtypes = [P]
        L.scr_ctx_bytes_in_use.restype = C.c_int64
        L.amg_setup.argtypes = [P, C.c_int, C.POINTER(ScrBsr), P, C.POINTER(AmgOpts), P, C.POINTER(P)]
        L.scr_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), P, C.POINTER(Stats)]
        L.mesh_motion_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), P, C.POINTER(Stats)]
        L.scr_handle_destroy.argtypes = [P]
        L.scr_handle_bytes.argtypes = [P]
        L.scr_handle_bytes.restype = C.c_int64
        L.scr_footprint_estimate.argtypes = [C.c_int, C.c_int64, C.c_int64, C.POINTER(AmgOpts), C.POINTER(SolveOpts)]
        L.scr_footprint_estimate.restype = C.c_int64
        L.scr_status_str.argtypes = [C.c_int]
        L.scr_status_str.restype = C.c_char_p
        L.scr_last_error.restype = C.c_char_p
        L.scr_hier_levels.argtypes = [P, C.c_int, C.POINTER(C.c_int)]
        L.scr_hier_level_info.argtypes = [P, C.c_int, C.c_int, P, C.POINTER(C.c_double)]
        L.scr_hier_level_copy.argtypes = [P, C.c_int, C.c_int, C.c_int, P]
        L.scr_matrix_copy.argtypes = [P, C.c_int, C.c_int, P, P]
        L.scr_apply.argtypes = [P, C.c_int, P, P, C.POINTER(SolveOpts), P]
        L.scr_ctx_profile.argtypes = [P, C.c_int]
        L.scr_ctx_profile_read.argtypes = [P, P, P, P]
        for f in ("amg_setup", "scr_solve", "mesh_motion_solve", "scr_handle_destroy", "scr_ctx_create",
                  "scr_hier_levels", "scr_hier_level_info", "scr_hier_level_copy", "scr_matrix_copy", "scr_apply",
                  "scr_ctx_profile", "scr_ctx_profile_read"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(status, allow=(SCR_OK,)):
    if status not in allow:
        raise ScrError(status, lib().scr_last_error().decode())
    return status


def amg_opts(**kw) -> AmgOpts:
    o = AmgOpts()
    lib().scr_default_amg_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def solve_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().scr_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.ptr = P()
        _check(lib().scr_ctx_create(device, hbm_budget, C.byref(self.ptr)))

    def bytes_in_use(self) -> int:
        return lib().scr_ctx_bytes_in_use(self.ptr)

    def profile(self, kernel: int):
        _check(lib().scr_ctx_profile(self.ptr, kernel))

    def profile_read(self):
        """(launches, total_ms, algorithmic_bytes) of the profiled kernel since the last read."""
        n = C.c_int64(); ms = C.c_double(); by = C.c_double()
        _check(lib().scr_ctx_profile_read(self.ptr, C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def destroy(self):
        if self.ptr:
            lib().scr_ctx_destroy(self.ptr)
            self.ptr = P()


class Handle:
    def __init__(self, ptr, kind, n_brows):
        self.ptr, self.kind, self.n_brows = ptr, kind, n_brows

    def destroy(self):
        if self.ptr:
            _check(lib().scr_handle_destroy(self.ptr))
            self.ptr = P()

    def bytes(self) -> int:
        return lib().scr_handle_bytes(self.ptr)

    # ---- inspection
    def hier_levels(self, which: int) -> int:
        n = C.c_int()
        _check(lib().scr_hier_levels(self.ptr, which, C.byref(n)))
        return n.value

    def hier_level_info(self, which: int, level: int) -> dict:
        info = np.zeros(8, np.int64)
        lam = C.c_double()
        _check(lib().scr_hier_level_info(self.ptr, which, level, info.ctypes.data_as(P), C.byref(lam)))
        nr, b, k, nnzA, nagg, nnzP, nnzR, ncoarse = (int(v) for v in info)
        return dict(nr=nr, b=b, k=k, nnzA=nnzA, nagg=nagg, nnzP=nnzP, nnzR=nnzR, ncoarse=ncoarse, lam=lam.value)

    FIELDS = {"A.rp": 0, "A.ci": 1, "A.v": 2, "agg": 3, "P.rp": 4, "P.ci": 5, "P.v": 6, "R.rp": 7, "R.ci": 8,
              "R.v": 9, "strong": 10, "dead": 11, "Dinv": 12, "B": 13}

    def hier_level_copy(self, which: int, level: int, field: str) -> np.ndarray:
        i = self.hier_level_info(which, level)
        f = self.FIELDS[field]
        shapes = {0: ((i["nr"] + 1,), np.int32), 1: ((i["nnzA"],), np.int32),
                  2: ((i["nnzA"], i["b"], i["b"]), np.float64), 3: ((i["nr"],), np.int32),
                  4: ((i["nr"] + 1,), np.int32), 5: ((i["nnzP"],), np.int32),
                  6: ((i["nnzP"], i["b"], i["k"]), np.float64), 7: ((i["nagg"] + 1,), np.int32),
                  8: ((i["nnzR"],), np.int32), 9: ((i["nnzR"], i["k"], i["b"]), np.float64),
                  10: ((i["nnzA"],), np.uint8), 11: ((i["nagg"] * i["k"],), np.uint8),
                  12: ((i["nr"], i["b"], i["b"]), np.float64), 13: ((i["nr"] * i["b"], i["k"]), np.float64)}
        shape, dt = shapes[f]
        out = np.empty(shape, dt)
        _check(lib().scr_hier_level_copy(self.ptr, which, level, f, out.ctypes.data_as(P)))
        return out

    def matrix_copy(self, which: str):
        w = {"A": 0, "G": 1, "D": 2, "C": 3, "Shat": 4}[which]
        info = np.zeros(4, np.int64)
        _check(lib().scr_matrix_copy(self.ptr, w, 0, None, info.ctypes.data_as(P)))
        nr, nnz, br, bc = (int(v) for v in info)
        rp = np.empty(nr + 1, np.int32); ci = np.empty(nnz, np.int32); v = np.empty((nnz, br, bc))
        for f, a in ((0, rp), (1, ci), (2, v)):
            _check(lib().scr_matrix_copy(self.ptr, w, f, a.ctypes.data_as(P), info.ctypes.data_as(P)))
        return rp, ci, v


def amg_setup(ctx: Context, kind: int, row_ptr, col_idx, val, coords=None, opts: AmgOpts | None = None,
              stream=None) -> Handle:
    import torch
    n = row_ptr.numel() - 1
    bs = 4 if kind == SCR_SYSTEM else 1
    K = ScrBsr(n_brows=n, bs=bs, nnzb=col_idx.numel(), row_ptr=_dev(row_ptr, torch.int32, "row_ptr"),
               col_idx=_dev(col_idx, torch.int32, "col_idx"), val=_dev(val, torch.float64, "val"))
    cp = _dev(coords, torch.float64, "coords") if coords is not None else None
    h = P()
    _check(lib().amg_setup(ctx.ptr, kind, C.byref(K), cp, C.byref(opts) if opts else None, _stream(stream),
                           C.byref(h)))
    return Handle(h, kind, n)


def scr_solve(h: Handle, b, x, opts: SolveOpts | None = None, stream=None):
    import torch
    st = Stats()
    rc = _check(lib().scr_solve(h.ptr, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"),
                                C.byref(opts) if opts else None, _stream(stream), C.byref(st)),
                allow=(SCR_OK, SCR_NOT_CONVERGED))
    return rc, st.as_dict()


def mesh_motion_solve(h: Handle, b, x, opts: SolveOpts | None = None, stream=None):
    import torch
    st = Stats()
    rc = _check(lib().mesh_motion_solve(h.ptr, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"),
                                        C.byref(opts) if opts else None, _stream(stream), C.byref(st)),
                allow=(SCR_OK, SCR_NOT_CONVERGED))
    return rc, st.as_dict()


OPS = {"K": 0, "A": 1, "VA": 2, "VS": 3, "S": 4, "SCR": 5, "G": 6, "D": 7, "C": 8, "Shat": 9, "L": 10, "VL": 11}


def scr_apply(h: Handle, op: str, x, y, opts: SolveOpts | None = None, stream=None):
    import torch
    _check(lib().scr_apply(h.ptr, OPS[op], _dev(x, torch.float64, "x"), _dev(y, torch.float64, "y"),
                           C.byref(opts) if opts else None, _stream(stream)))


def footprint_estimate(kind: int, n_brows: int, nnzb: int, amg: AmgOpts | None = None,
                       solve: SolveOpts | None = None) -> int:
    return lib().scr_footprint_estimate(kind, n_brows, nnzb, C.byref(amg) if amg else None,
                                        C.byref(solve) if solve else None)
