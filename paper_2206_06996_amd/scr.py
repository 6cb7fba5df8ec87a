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
SCR_FP64, SCR_MIXED, SCR_MIXED_FP32_INNER = 0, 1, 2
SCR_SMOOTH_JACOBI, SCR_SMOOTH_CHEBYSHEV = 0, 1
SCR_AMG_SA, SCR_AMG_CLASSICAL = 0, 1

EXPORTED = ["scr_default_amg_opts", "scr_default_solve_opts", "scr_ctx_create", "scr_ctx_destroy",
            "scr_ctx_bytes_in_use", "scr_handle_peak_bytes", "mesh_motion_solve_noalloc", "amg_setup", "amg_update", "scr_set_outlets", "scr_solve", "mesh_motion_solve", "scr_handle_destroy",
            "scr_handle_bytes", "scr_footprint_estimate", "scr_status_str", "scr_last_error", "scr_hier_levels",
            "scr_hier_level_info", "scr_hier_level_copy", "scr_matrix_copy", "scr_apply", "scr_ctx_profile",
            "scr_ctx_profile_read", "srv_create", "srv_submit", "srv_poll", "srv_wait", "srv_drain",
            "srv_destroy", "scr_assembler_create", "scr_assemble_tangent", "scr_assembler_nnzb",
            "scr_assembler_nbrows", "scr_assembler_destroy", "scr_default_corrector_opts", "scr_stepper_create",
            "scr_stepper_state", "scr_step", "scr_stepper_destroy"]
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
                ("max_levels", C.c_int), ("max_coarse_ratio", C.c_double), ("seed", C.c_uint64),
                ("schur_diag", C.c_int), ("schur_cheb_degree", C.c_int), ("schur_cheb_ratio", C.c_double),
                ("amg_type", C.c_int), ("cl_theta", C.c_double), ("trunc", C.c_double), ("pmax", C.c_int),
                ("agg_levels", C.c_int), ("l1_gs", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_A", C.c_double), ("tol_S", C.c_double), ("tol_I", C.c_double),
                ("max_it", C.c_int), ("max_it_A", C.c_int), ("max_it_S", C.c_int), ("max_it_I", C.c_int),
                ("restart", C.c_int), ("restart_inner", C.c_int), ("use_x0", C.c_int), ("flexible_cg", C.c_int),
                ("precond", C.c_int)]


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


class ScrRequest(C.Structure):
    _fields_ = [("K", ScrBsr), ("coords", P), ("n_rhs", C.c_int), ("b", C.POINTER(P)), ("x", C.POINTER(P)),
                ("L", C.POINTER(ScrBsr)), ("bm", C.POINTER(P)), ("xm", C.POINTER(P)), ("vals", C.POINTER(P)),
                ("tangent", P), ("u", C.POINTER(P))]


class SrvResult(C.Structure):
    _fields_ = [("status", C.c_int), ("n_solves", C.c_int64), ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("footprint", C.c_int64),
                ("device_bytes", C.c_int64), ("last", Stats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "last"}
        d["last"] = self.last.as_dict()
        return d


class TangentParams(C.Structure):
    """scr_tangent_params: physical constants of the tangent assembly."""
    _fields_ = [("rho_f", C.c_double), ("mu_f", C.c_double), ("rho_s", C.c_double), ("E_s", C.c_double),
                ("nu_s", C.c_double), ("dt", C.c_double), ("rho_inf", C.c_double), ("terms", C.c_int32),
                ("vms_dt_coupling", C.c_int32)]


class CorrectorOpts(C.Structure):
    _fields_ = [("max_correctors", C.c_int32), ("tol_R", C.c_double), ("tol_A", C.c_double),
                ("mesh_tol", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("correctors", C.c_int32), ("converged", C.c_int32), ("res0", C.c_double), ("res", C.c_double),
                ("linear_its", C.c_int64), ("mesh_its", C.c_int64), ("resetups", C.c_int32), ("t_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SCR_STATE = {"y": 0, "ydot": 1, "u_solid": 2, "udot_solid": 3, "u_mesh": 4, "v_mesh": 5}


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
        L.amg_update.argtypes = [P, C.POINTER(ScrBsr), P, P]
        L.scr_set_outlets.argtypes = [P, C.c_int, P, P, P, P, P]
        L.scr_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), P, C.POINTER(Stats)]
        L.mesh_motion_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), P, C.POINTER(Stats)]
        L.mesh_motion_solve_noalloc.argtypes = [P, P, P, C.POINTER(SolveOpts), P, C.POINTER(Stats)]
        L.scr_handle_destroy.argtypes = [P]
        L.scr_handle_bytes.argtypes = [P]
        L.scr_handle_bytes.restype = C.c_int64
        L.scr_handle_peak_bytes.argtypes = [P]
        L.scr_handle_peak_bytes.restype = C.c_int64
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
        L.srv_create.argtypes = [P, C.c_int, C.c_int64, C.POINTER(AmgOpts), C.POINTER(SolveOpts), C.POINTER(P)]
        L.srv_submit.argtypes = [P, C.POINTER(ScrRequest), C.POINTER(C.c_int64)]
        L.srv_poll.argtypes = [P, C.c_int64, C.POINTER(C.c_int), C.POINTER(SrvResult)]
        L.srv_wait.argtypes = [P, C.c_int64, C.POINTER(SrvResult)]
        L.srv_drain.argtypes = [P, C.POINTER(C.c_int)]
        L.srv_destroy.argtypes = [P]
        L.srv_destroy.restype = None
        L.scr_assembler_create.argtypes = [P, C.c_int64, P, P, P, C.c_int64, P, P, P, P,
                                           C.POINTER(TangentParams), P, C.POINTER(P)]
        L.scr_assemble_tangent.argtypes = [P, P, P, P]
        L.scr_assembler_nnzb.argtypes = [P]
        L.scr_assembler_nnzb.restype = C.c_int64
        L.scr_assembler_nbrows.argtypes = [P]
        L.scr_assembler_nbrows.restype = C.c_int64
        L.scr_assembler_destroy.argtypes = [P]
        L.scr_default_corrector_opts.argtypes = [C.POINTER(CorrectorOpts)]
        L.scr_default_corrector_opts.restype = None
        L.scr_stepper_create.argtypes = [P, P, C.POINTER(ScrBsr), P, P, P, P, P, C.c_double, C.POINTER(AmgOpts),
                                         C.POINTER(SolveOpts), C.POINTER(CorrectorOpts), P, C.POINTER(P)]
        L.scr_stepper_state.argtypes = [P, C.c_int, P, C.c_int, P]
        L.scr_step.argtypes = [P, C.c_double, P, P, C.POINTER(StepStats)]
        L.scr_stepper_destroy.argtypes = [P]
        for f in ("amg_setup", "amg_update", "scr_set_outlets", "scr_solve", "mesh_motion_solve",
                  "mesh_motion_solve_noalloc", "scr_handle_destroy", "scr_ctx_create",
                  "scr_hier_levels", "scr_hier_level_info", "scr_hier_level_copy", "scr_matrix_copy", "scr_apply",
                  "scr_ctx_profile", "scr_ctx_profile_read", "srv_create", "srv_submit", "srv_poll", "srv_wait",
                  "srv_drain", "scr_assembler_create", "scr_assemble_tangent", "scr_assembler_destroy",
                  "scr_stepper_create", "scr_stepper_state", "scr_step", "scr_stepper_destroy"):
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

    def peak_bytes(self) -> int:
        return lib().scr_handle_peak_bytes(self.ptr)

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
              "R.v": 9, "strong": 10, "dead": 11, "Dinv": 12, "B": 13, "func": 15}

    def hier_level_copy(self, which: int, level: int, field: str) -> np.ndarray:
        i = self.hier_level_info(which, level)
        f = self.FIELDS[field]
        shapes = {0: ((i["nr"] + 1,), np.int32), 1: ((i["nnzA"],), np.int32),
                  2: ((i["nnzA"], i["b"], i["b"]), np.float64), 3: ((i["nr"],), np.int32),
                  4: ((i["nr"] + 1,), np.int32), 5: ((i["nnzP"],), np.int32),
                  6: ((i["nnzP"], i["b"], i["k"]), np.float64), 7: ((i["nagg"] + 1,), np.int32),
                  8: ((i["nnzR"],), np.int32), 9: ((i["nnzR"], i["k"], i["b"]), np.float64),
                  10: ((i["nnzA"],), np.uint8), 11: ((i["nagg"] * i["k"],), np.uint8),
                  12: ((i["nr"], i["b"], i["b"]), np.float64), 13: ((i["nr"] * i["b"], i["k"]), np.float64),
                  15: ((i["nr"],), np.uint8)}
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


def amg_update(h: Handle, row_ptr, col_idx, val, coords=None, stream=None):
    """Numeric re-setup of h for new values on the same pattern (and new coordinates, optional)."""
    import torch
    bs = 4 if h.kind == SCR_SYSTEM else 1
    K = ScrBsr(n_brows=row_ptr.numel() - 1, bs=bs, nnzb=col_idx.numel(),
               row_ptr=_dev(row_ptr, torch.int32, "row_ptr"), col_idx=_dev(col_idx, torch.int32, "col_idx"),
               val=_dev(val, torch.float64, "val"))
    cp = _dev(coords, torch.float64, "coords") if coords is not None else None
    _check(lib().amg_update(h.ptr, C.byref(K), cp, _stream(stream)))


def set_outlets(h: Handle, outlets, m, stream=None):
    """Outlet resistance coupling: outlets = [(block rows, a (n, 3)), ...] (numpy arrays), m =
    one coefficient per outlet; an empty list removes the coupling."""
    import torch
    n = len(outlets)
    off = np.zeros(n + 1, np.int64)
    for k, (blk, _) in enumerate(outlets):
        off[k + 1] = off[k] + len(blk)
    mm = np.ascontiguousarray(np.asarray(m, np.float64).reshape(-1)[:n] if n else np.zeros(1))
    blk = a = None
    if n:
        blk = torch.from_numpy(np.ascontiguousarray(np.concatenate([np.asarray(b) for b, _ in outlets]), np.int32)).to("cuda")
        a = torch.from_numpy(np.ascontiguousarray(np.concatenate([np.asarray(v).reshape(-1) for _, v in outlets]),
                                                  np.float64)).to("cuda")
    _check(lib().scr_set_outlets(h.ptr, n, off.ctypes.data_as(P), None if blk is None else _dev(blk, torch.int32, "blk"),
                                 None if a is None else _dev(a, torch.float64, "a"), mm.ctypes.data_as(P),
                                 _stream(stream)))


def tangent_params(**kw) -> TangentParams:
    """Defaults: every term, no c_t coupling in D; the physical constants must be given."""
    t = TangentParams(terms=63, vms_dt_coupling=0)
    for k, v in kw.items():
        setattr(t, k, v)
    return t


class Assembler:
    def __init__(self, ptr, n_brows, nnzb):
        self.ptr, self.n_brows, self.nnzb = ptr, n_brows, nnzb

    def destroy(self):
        if self.ptr:
            lib().scr_assembler_destroy(self.ptr)
            self.ptr = P()


def scr_assembler_create(ctx: Context, tv, tp, solid, row_ptr, col_idx, coords, mask, params: TangentParams,
                         stream=None) -> Assembler:
    """tv, tp: (n_tets, 4) int32; solid: n_tets uint8; row_ptr, col_idx: int32 pattern; coords:
    (n_brows, 3) FP64; mask: 4 n_brows uint8 (all device tensors)."""
    import torch
    a = P()
    n = row_ptr.numel() - 1
    nt = tv.shape[0] if tv.dim() == 2 else -1
    if tv.shape != (nt, 4) or tp.shape != (nt, 4) or solid.numel() != nt:
        raise ValueError("tv and tp must be (n_tets, 4) and solid n_tets long")
    if coords.numel() != 3 * n or mask.numel() != 4 * n:
        raise ValueError("coords must hold 3 n_brows and mask 4 n_brows values")
    if n < 1 or col_idx.numel() != int(row_ptr[-1].item()):
        raise ValueError("col_idx must hold row_ptr[n_brows] entries")
    _check(lib().scr_assembler_create(ctx.ptr, tv.shape[0], _dev(tv, torch.int32, "tv"), _dev(tp, torch.int32, "tp"),
                                      _dev(solid, torch.uint8, "solid"), n, _dev(row_ptr, torch.int32, "row_ptr"),
                                      _dev(col_idx, torch.int32, "col_idx"), _dev(coords, torch.float64, "coords"),
                                      _dev(mask, torch.uint8, "mask"), C.byref(params), _stream(stream), C.byref(a)))
    return Assembler(a, n, lib().scr_assembler_nnzb(a))


def scr_assemble_tangent(a: Assembler, u, val, stream=None):
    """val (16 nnzb FP64, device) = the tangent at the advective velocity u ((n_brows, 3) FP64
    device tensor, or None for the tangent at rest)."""
    import torch
    if val.numel() != 16 * a.nnzb:
        raise ValueError("val must hold 16 * nnzb values")
    if u is not None and u.numel() != 3 * a.n_brows:
        raise ValueError("u must hold 3 * n_brows values")
    _check(lib().scr_assemble_tangent(a.ptr, None if u is None else _dev(u, torch.float64, "u"),
                                      _dev(val, torch.float64, "val"), _stream(stream)))


def corrector_opts(**kw) -> CorrectorOpts:
    o = CorrectorOpts()
    lib().scr_default_corrector_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Stepper:
    """The predictor multi-corrector time stepper (scr_stepper_*)."""

    def __init__(self, ptr, n_brows, n_mesh):
        self.ptr, self.n_brows, self.n_mesh = ptr, n_brows, n_mesh

    def _size(self, field):
        return 4 * self.n_brows if field < 2 else 3 * self.n_brows if field < 4 else 3 * self.n_mesh

    def state(self, field: str, out=None, stream=None):
        """Copy a field of the state at t_n into out (a new FP64 device tensor if None)."""
        import torch
        f = SCR_STATE[field]
        if out is None:
            out = torch.empty(self._size(f), dtype=torch.float64, device="cuda")
        if out.numel() != self._size(f):
            raise ValueError(f"{field} holds {self._size(f)} values")
        _check(lib().scr_stepper_state(self.ptr, f, _dev(out, torch.float64, field), 0, _stream(stream)))
        return out

    def set_state(self, field: str, src, stream=None):
        import torch
        f = SCR_STATE[field]
        if src.numel() != self._size(f):
            raise ValueError(f"{field} holds {self._size(f)} values")
        _check(lib().scr_stepper_state(self.ptr, f, _dev(src, torch.float64, field), 1, _stream(stream)))

    def step(self, dt: float, f=None, stream=None):
        """One time step; returns (status, stats dict)."""
        import torch
        if f is not None and f.numel() != 3 * self.n_brows:
            raise ValueError("f must hold 3 * n_brows values")
        st = StepStats()
        rc = _check(lib().scr_step(self.ptr, float(dt), None if f is None else _dev(f, torch.float64, "f"),
                                   _stream(stream), C.byref(st)), allow=(SCR_OK, SCR_NOT_CONVERGED))
        return rc, st.as_dict()

    def destroy(self):
        if self.ptr:
            lib().scr_stepper_destroy(self.ptr)
            self.ptr = P()


def scr_stepper_create(ctx: Context, a: Assembler, L_row_ptr, L_col_idx, L_val, L_full, mesh_mask, blk_of_phys,
                       solid_rows, coords, dt0: float, amg: AmgOpts | None = None, solve: SolveOpts | None = None,
                       copts: CorrectorOpts | None = None, stream=None) -> Stepper:
    """L_*: the eliminated mesh Laplacian (CSR, device); L_full: its values before the elimination;
    mesh_mask: n_L uint8; blk_of_phys: n_L int32; solid_rows: n_brows uint8; coords: n_brows x 3."""
    import torch
    nL = L_row_ptr.numel() - 1
    if L_val.numel() != L_col_idx.numel() or L_full.numel() != L_col_idx.numel():
        raise ValueError("L_val and L_full must hold nnz(L) values")
    if mesh_mask.numel() != nL or blk_of_phys.numel() != nL:
        raise ValueError("mesh_mask and blk_of_phys must hold n_L entries")
    if solid_rows.numel() != a.n_brows or coords.numel() != 3 * a.n_brows:
        raise ValueError("solid_rows must hold n_brows and coords 3 n_brows entries")
    Lb = _bsr(L_row_ptr, L_col_idx, L_val, 1)
    s = P()
    _check(lib().scr_stepper_create(ctx.ptr, a.ptr, C.byref(Lb), _dev(L_full, torch.float64, "L_full"),
                                    _dev(mesh_mask, torch.uint8, "mesh_mask"),
                                    _dev(blk_of_phys, torch.int32, "blk_of_phys"),
                                    _dev(solid_rows, torch.uint8, "solid_rows"), _dev(coords, torch.float64, "coords"),
                                    float(dt0), C.byref(amg) if amg else None, C.byref(solve) if solve else None,
                                    C.byref(copts) if copts else None, _stream(stream), C.byref(s)))
    return Stepper(s, a.n_brows, nL)


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


def mesh_motion_solve_noalloc(h: Handle, b, x, opts: SolveOpts | None = None, stream=None):
    """mesh_motion_solve with the CG workspace in the library's static device scratch."""
    import torch
    st = Stats()
    rc = _check(lib().mesh_motion_solve_noalloc(h.ptr, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"),
                                                C.byref(opts) if opts else None, _stream(stream), C.byref(st)),
                allow=(SCR_OK, SCR_NOT_CONVERGED))
    return rc, st.as_dict()


OPS = {"K": 0, "A": 1, "VA": 2, "VS": 3, "S": 4, "SCR": 5, "G": 6, "D": 7, "C": 8, "Shat": 9, "L": 10, "VL": 11,
       "SIMPLE": 12, "d": 13}
SCR_DIAG_A, SCR_DIAG_ABSROWSUM = 0, 1
SCR_PRECOND_SCR, SCR_PRECOND_SIMPLE = 0, 1


def scr_apply(h: Handle, op: str, x, y, opts: SolveOpts | None = None, stream=None):
    import torch
    _check(lib().scr_apply(h.ptr, OPS[op], _dev(x, torch.float64, "x"), _dev(y, torch.float64, "y"),
                           C.byref(opts) if opts else None, _stream(stream)))


def footprint_estimate(kind: int, n_brows: int, nnzb: int, amg: AmgOpts | None = None,
                       solve: SolveOpts | None = None) -> int:
    return lib().scr_footprint_estimate(kind, n_brows, nnzb, C.byref(amg) if amg else None,
                                        C.byref(solve) if solve else None)


def _bsr(row_ptr, col_idx, val, bs):
    import torch
    return ScrBsr(n_brows=row_ptr.numel() - 1, bs=bs, nnzb=col_idx.numel(),
                  row_ptr=_dev(row_ptr, torch.int32, "row_ptr"), col_idx=_dev(col_idx, torch.int32, "col_idx"),
                  val=_dev(val, torch.float64, "val"))


class Server:
    """Continuous-batching server (srv_* in scr.h).  submit() keeps references to the tensors of
    each request until it is waited for."""

    def __init__(self, ctx: Context, max_slots: int = 4, hbm_budget: int = 0, amg: AmgOpts | None = None,
                 solve: SolveOpts | None = None):
        self.ptr = P()
        self._keep = {}
        _check(lib().srv_create(ctx.ptr, max_slots, hbm_budget, C.byref(amg) if amg else None,
                                C.byref(solve) if solve else None, C.byref(self.ptr)))

    def submit(self, K, coords, bs, xs, L=None, bms=None, xms=None, vals=None, tangent=None, us=None) -> int:
        """K = (row_ptr, col_idx, val) tensors of the 4x4 system; bs/xs lists of RHS/output tensors;
        L = (row_ptr, col_idx, val) of the mesh Laplacian with bms/xms lists (optional); vals = a
        list with one entry per correction: None (keep the previous tangent) or the K values of
        that correction on K's pattern (the first entry is ignored).  tangent = an Assembler on K's
        pattern with us = one advective velocity per correction (a (n_brows, 3) tensor or None):
        the tangents are then assembled on the device (the first at us[0], None = at rest)."""
        import torch
        n = len(bs)
        barr = (P * n)(*[_dev(b, torch.float64, "b") for b in bs])
        xarr = (P * n)(*[_dev(x, torch.float64, "x") for x in xs])
        req = ScrRequest(K=_bsr(*K, 4), coords=_dev(coords, torch.float64, "coords"), n_rhs=n, b=barr, x=xarr)
        keep = [K, coords, bs, xs, barr, xarr]
        if L is not None:
            Lb = _bsr(*L, 1)
            bmarr = (P * n)(*[_dev(b, torch.float64, "bm") for b in bms])
            xmarr = (P * n)(*[_dev(x, torch.float64, "xm") for x in xms])
            req.L = C.pointer(Lb); req.bm = bmarr; req.xm = xmarr
            keep += [L, bms, xms, Lb, bmarr, xmarr]
        if vals is not None:
            varr = (P * n)(*[None if (v is None or c == 0) else _dev(v, torch.float64, "vals")
                             for c, v in enumerate(vals)])
            req.vals = varr
            keep += [vals, varr]
        if tangent is not None:
            req.tangent = tangent.ptr
            keep.append(tangent)
            if us is not None:
                for u in us:
                    if u is not None and u.numel() != 3 * tangent.n_brows:
                        raise ValueError("each u must hold 3 * n_brows values")
                uarr = (P * n)(*[None if u is None else _dev(u, torch.float64, "u") for u in us])
                req.u = uarr
                keep += [us, uarr]
        rid = C.c_int64()
        _check(lib().srv_submit(self.ptr, C.byref(req), C.byref(rid)))
        self._keep[rid.value] = keep
        return rid.value

    def poll(self, rid: int):
        done = C.c_int(); res = SrvResult()
        _check(lib().srv_poll(self.ptr, rid, C.byref(done), C.byref(res)))
        return (res.as_dict() if done.value else None)

    def wait(self, rid: int) -> dict:
        res = SrvResult()
        _check(lib().srv_wait(self.ptr, rid, C.byref(res)))
        self._keep.pop(rid, None)
        return res.as_dict()

    def drain(self) -> int:
        m = C.c_int()
        _check(lib().srv_drain(self.ptr, C.byref(m)))
        return m.value

    def destroy(self):
        if self.ptr:
            lib().srv_destroy(self.ptr)
            self.ptr = P()
            self._keep.clear()
