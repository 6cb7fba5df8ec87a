"""FP64 CPU oracle of the SCR+AMG linear-solve path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  The GPU library never links, loads or calls it, and the two share no code; the
only common dependency is the seeded input generator ``synth``.

The C source is ``oracle/oracle.c`` (plain loops, FP64, built with ``-ffp-contract=off`` so that
the strength predicate is evaluated without fused multiply-adds, as in its definition).  OpenMP
splits only loops with independent iterations and the dot products use fixed chunks, so every
result is the same bit for bit for any ``OMP_NUM_THREADS``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None
P = C.c_void_p


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-fopenmp", "-ffp-contract=off", src,
                    "-o", _SO + ".tmp", "-lm"], check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class AmgOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("smoother", C.c_int), ("cheb_degree", C.c_int),
                ("cheb_ratio", C.c_double), ("jacobi_sweeps", C.c_int), ("coarse_max", C.c_int),
                ("max_levels", C.c_int), ("max_coarse_ratio", C.c_double), ("seed", C.c_uint64),
                ("schur_diag", C.c_int), ("schur_cheb_degree", C.c_int), ("schur_cheb_ratio", C.c_double),
                ("amg_type", C.c_int), ("cl_theta", C.c_double), ("trunc", C.c_double), ("pmax", C.c_int),
                ("hmis_domain", C.c_int), ("gs_domain", C.c_int), ("agg_levels", C.c_int),
                ("l1_gs", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_A", C.c_double), ("tol_S", C.c_double), ("tol_I", C.c_double),
                ("max_it", C.c_int), ("max_it_A", C.c_int), ("max_it_S", C.c_int), ("max_it_I", C.c_int),
                ("restart", C.c_int), ("restart_inner", C.c_int), ("use_x0", C.c_int),
                ("flexible_cg", C.c_int), ("precond", C.c_int)]


class ScrStats(C.Structure):
    _fields_ = [("outer_it", C.c_int), ("rel_res_true", C.c_double), ("calls_A", C.c_int64),
                ("its_A", C.c_int64), ("calls_S", C.c_int64), ("its_S", C.c_int64),
                ("calls_I", C.c_int64), ("its_I", C.c_int64), ("vcycles_A", C.c_int64),
                ("vcycles_S", C.c_int64), ("converged", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def amg_opts(**kw) -> AmgOpts:
    """Defaults: smoothed aggregation with theta=0.08 (halved per level), Chebyshev degree 4 on
    [lam/30, lam], coarse solve below 1024 unknowns, at most 10 levels, stop if coarsening is
    slower than 0.8.  amg_type=1: classical AMG with the paper's settings (strength 0.5, HMIS on
    domains of 256 rows, aggressive two-stage coarsening on the first two levels, extended+i truncated
    at 0.3 with at most 5 entries, hybrid Gauss-Seidel on domains of 64 rows)."""
    o = AmgOpts(theta=0.08, smoother=1, cheb_degree=4, cheb_ratio=30.0, jacobi_sweeps=2,
                coarse_max=1024, max_levels=10, max_coarse_ratio=0.8, seed=0, schur_diag=0,
                schur_cheb_degree=-1, schur_cheb_ratio=100.0, amg_type=0, cl_theta=0.5, trunc=0.3, pmax=5,
                hmis_domain=256, gs_domain=64, agg_levels=2, l1_gs=1)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def solve_opts(**kw) -> SolveOpts:
    """Defaults: outer delta 1e-8; delta_A = delta_S = delta_I = 1e-3 and 200 iterations at
    every level (the paper's solver-settings table, Sec. 6); restarts 50 outer / 30 inner."""
    o = SolveOpts(tol=1e-8, tol_A=1e-3, tol_S=1e-3, tol_I=1e-3, max_it=200, max_it_A=200,
                  max_it_S=200, max_it_I=200, restart=50, restart_inner=30, use_x0=0, flexible_cg=0,
                  precond=0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_dense_solve.argtypes = [C.c_int64, P, P, P]
        L.orc_dense_solve.restype = C.c_int
        L.orc_bsr_spmv.argtypes = [C.c_int64, C.c_int64, C.c_int, C.c_int, P, P, P, P, P]
        L.orc_strength.argtypes = [C.c_int64, C.c_int, P, P, P, C.c_double, P, P]
        L.orc_mis_key.argtypes = [C.c_uint64, C.c_int, C.c_int64]
        L.orc_mis_key.restype = C.c_uint64
        L.orc_num_threads.restype = C.c_int
        L.orc_mis2.argtypes = [C.c_int64, P, P, P, P, C.c_uint64, C.c_int, P]
        L.orc_aggregate.argtypes = [C.c_int64, P, P, P, P, P, C.c_uint64, C.c_int, P]
        L.orc_aggregate.restype = C.c_int64
        L.orc_amg_create.argtypes = [C.c_int64, C.c_int, P, P, P, P, C.c_int, C.POINTER(AmgOpts), C.POINTER(P)]
        L.orc_amg_create.restype = C.c_int
        L.orc_amg_free.argtypes = [P]
        L.orc_amg_vcycle.argtypes = [P, P, P]
        L.orc_amg_smooth.argtypes = [P, C.c_int, P, P, C.c_int]
        L.orc_amg_nlevels.argtypes = [P]
        L.orc_amg_nlevels.restype = C.c_int
        L.orc_amg_level_info.argtypes = [P, C.c_int, P, P]
        L.orc_amg_level_get.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_amg_level_get.restype = C.c_int
        L.orc_scr_create.argtypes = [C.c_int64, P, P, P, P, C.POINTER(AmgOpts), C.POINTER(P)]
        L.orc_scr_create.restype = C.c_int
        L.orc_scr_free.argtypes = [P]
        L.orc_scr_amg.argtypes = [P, C.c_int]
        L.orc_scr_amg.restype = P
        L.orc_scr_matrix.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_scr_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), C.POINTER(ScrStats)]
        L.orc_scr_solve.restype = C.c_int
        L.orc_scr_apply.argtypes = [P, C.c_int, P, P, C.POINTER(SolveOpts)]
        L.orc_scr_apply.restype = C.c_int
        L.orc_amg_update.argtypes = [P, P, P]
        L.orc_amg_update.restype = C.c_int
        L.orc_scr_update.argtypes = [P, P, P]
        L.orc_scr_update.restype = C.c_int
        L.orc_scr_set_outlets.argtypes = [P, C.c_int, P, P, P, P]
        L.orc_scr_set_outlets.restype = C.c_int
        L.orc_mesh_update.argtypes = [P, P]
        L.orc_mesh_update.restype = C.c_int
        L.orc_mesh_create.argtypes = [C.c_int64, P, P, P, C.POINTER(AmgOpts), C.POINTER(P)]
        L.orc_mesh_create.restype = C.c_int
        L.orc_mesh_free.argtypes = [P]
        L.orc_mesh_amg.argtypes = [P]
        L.orc_mesh_amg.restype = P
        L.orc_mesh_solve.argtypes = [P, P, P, C.c_double, C.c_int, C.c_int, P, P]
        L.orc_mesh_solve.restype = C.c_int
        L.orc_gmres.argtypes = [C.c_int64, C.c_int, P, P, P, P, P, P, C.c_double, C.c_int, C.c_int, P, P]
        L.orc_gmres.restype = C.c_int
        L.orc_cg.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_double, C.c_int, C.c_int, P, P]
        L.orc_cg.restype = C.c_int
        L.orc_cl_strength.argtypes = [C.c_int64, P, P, P, P, C.c_double, P]
        L.orc_cl_hmis.argtypes = [C.c_int64, P, P, P, C.c_int, C.c_uint64, C.c_int, P, P]
        L.orc_cl_hmis.restype = C.c_int
        L.orc_cl_extpi.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_double, C.c_int, P, P, P]
        L.orc_cl_extpi.restype = C.c_int64
        L.orc_cl_gs.argtypes = [C.c_int64, P, P, P, C.c_int, C.c_int, C.c_int, P, P, P]
        L.orc_cl_second_stage.argtypes = [C.c_int64, P, P, P, P, P, P, P]
        L.orc_cl_second_stage.restype = C.c_int64
        L.orc_cl_uniform.argtypes = [C.c_uint64, C.c_int, C.c_int64]
        L.orc_cl_uniform.restype = C.c_double
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(P)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def dense_solve(A, b):
    A = _c(A, np.float64); b = _c(b, np.float64)
    x = np.empty_like(b)
    rc = lib().orc_dense_solve(A.shape[0], _p(A), _p(b), _p(x))
    if rc:
        raise np.linalg.LinAlgError("zero pivot")
    return x


def bsr_spmv(rp, ci, val, x, ncols=None):
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64); x = _c(x, np.float64)
    nr = rp.size - 1
    br, bc = (val.shape[1], val.shape[2]) if val.ndim == 3 else (1, 1)
    nc = ncols if ncols is not None else x.size // bc
    y = np.empty(nr * br)
    lib().orc_bsr_spmv(nr, nc, br, bc, _p(rp), _p(ci), _p(val), _p(x), _p(y))
    return y


def strength(rp, ci, val, theta):
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64)
    nr = rp.size - 1
    b = val.shape[1] if val.ndim == 3 else 1
    flags = np.empty(ci.size, np.uint8); iso = np.empty(nr, np.uint8)
    lib().orc_strength(nr, b, _p(rp), _p(ci), _p(val), theta, _p(flags), _p(iso))
    return flags, iso


def num_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().orc_num_threads())


def mis_key(seed, level, i):
    return int(lib().orc_mis_key(seed, level, i))


def mis2(rp, ci, flags, iso, seed, level):
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); flags = _c(flags, np.uint8); iso = _c(iso, np.uint8)
    root = np.empty(rp.size - 1, np.uint8)
    lib().orc_mis2(rp.size - 1, _p(rp), _p(ci), _p(flags), _p(iso), seed, level, _p(root))
    return root


def aggregate(rp, ci, flags, iso, root, seed, level):
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); flags = _c(flags, np.uint8)
    iso = _c(iso, np.uint8); root = _c(root, np.uint8)
    agg = np.empty(rp.size - 1, np.int32)
    na = lib().orc_aggregate(rp.size - 1, _p(rp), _p(ci), _p(flags), _p(iso), _p(root), seed, level, _p(agg))
    return int(na), agg


def cl_strength(rp, ci, val, func, theta=0.5):
    """Classical strength flags (one per stored entry) of a scalar CSR matrix."""
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64); func = _c(func, np.uint8)
    S = np.empty(ci.size, np.uint8)
    lib().orc_cl_strength(rp.size - 1, _p(rp), _p(ci), _p(val), _p(func), theta, _p(S))
    return S


def cl_hmis(rp, ci, S, domain=256, seed=0, level=0):
    """HMIS C/F split: (cf, first) with 1 = C, -1 = F (first: the domain-wise first pass)."""
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); S = _c(S, np.uint8)
    nr = rp.size - 1
    cf = np.empty(nr, np.int8); first = np.empty(nr, np.int8)
    if lib().orc_cl_hmis(nr, _p(rp), _p(ci), _p(S), domain, seed, level, _p(cf), _p(first)):
        raise ValueError("pattern is not structurally symmetric")
    return cf, first


def cl_second_stage(rp, ci, S, cf):
    """The second-stage graph of aggressive coarsening on the C points of cf: (rp, ci, edge flags)
    in the numbering of the C points."""
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); S = _c(S, np.uint8); cf = _c(cf, np.int8)
    n1 = int((cf == 1).sum())
    grp = np.empty(n1 + 1, np.int32)
    nnz = lib().orc_cl_second_stage(rp.size - 1, _p(rp), _p(ci), _p(S), _p(cf), _p(grp), None, None)
    gci = np.empty(nnz, np.int32); gS = np.empty(nnz, np.uint8)
    lib().orc_cl_second_stage(rp.size - 1, _p(rp), _p(ci), _p(S), _p(cf), _p(grp), _p(gci), _p(gS))
    return grp, gci, gS


def cl_uniform(seed, level, i):
    return float(lib().orc_cl_uniform(seed, level, i))


def cl_extpi(rp, ci, val, func, S, cf, trunc=0.3, pmax=5):
    """Extended+i interpolation of a C/F split: (P.rp, P.ci, P.v), columns = coarse indices."""
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64); func = _c(func, np.uint8)
    S = _c(S, np.uint8); cf = _c(cf, np.int8)
    nr = rp.size - 1
    prp = np.empty(nr + 1, np.int32)
    nnz = lib().orc_cl_extpi(nr, _p(rp), _p(ci), _p(val), _p(func), _p(S), _p(cf), trunc, pmax, _p(prp), None, None)
    pci = np.empty(nnz, np.int32); pv = np.empty(nnz)
    lib().orc_cl_extpi(nr, _p(rp), _p(ci), _p(val), _p(func), _p(S), _p(cf), trunc, pmax, _p(prp), _p(pci), _p(pv))
    return prp, pci, pv


def cl_gs(rp, ci, val, b, x_old=None, domain=64, backward=False, l1=False):
    """One hybrid Gauss-Seidel sweep from x_old (None = zero); l1: the l1 form."""
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64); b = _c(b, np.float64)
    x = np.zeros_like(b)
    xo = None if x_old is None else _c(x_old, np.float64)
    lib().orc_cl_gs(rp.size - 1, _p(rp), _p(ci), _p(val), domain, int(backward), int(l1), _p(b),
                    None if xo is None else _p(xo), _p(x))
    return x


class Hierarchy:
    """Read access to one AMG hierarchy (owned by an Amg, Scr or Mesh object)."""

    FIELDS = {"A.rp": 0, "A.ci": 1, "A.v": 2, "agg": 3, "P.rp": 4, "P.ci": 5, "P.v": 6,
              "R.rp": 7, "R.ci": 8, "R.v": 9, "strong": 10, "dead": 11, "Dinv": 12, "B": 13, "Q": 14,
              "func": 15}

    def __init__(self, h, owner):
        self.h = h
        self._owner = owner

    @property
    def nlevels(self):
        return lib().orc_amg_nlevels(self.h)

    def info(self, l):
        info = np.zeros(8, np.int64); lam = np.zeros(1)
        lib().orc_amg_level_info(self.h, l, _p(info), _p(lam))
        nr, b, k, nnzA, nagg, nnzP, nnzR, ncoarse = (int(v) for v in info)
        return dict(nr=nr, b=b, k=k, nnzA=nnzA, nagg=nagg, nnzP=nnzP, nnzR=nnzR, ncoarse=ncoarse,
                    lam=float(lam[0]))

    def get(self, l, field):
        i = self.info(l)
        f = self.FIELDS[field]
        shapes = {0: ((i["nr"] + 1,), np.int32), 1: ((i["nnzA"],), np.int32),
                  2: ((i["nnzA"], i["b"], i["b"]), np.float64), 3: ((i["nr"],), np.int32),
                  4: ((i["nr"] + 1,), np.int32), 5: ((i["nnzP"],), np.int32),
                  6: ((i["nnzP"], i["b"], i["k"]), np.float64), 7: ((i["nagg"] + 1,), np.int32),
                  8: ((i["nnzR"],), np.int32), 9: ((i["nnzR"], i["k"], i["b"]), np.float64),
                  10: ((i["nnzA"],), np.uint8), 11: ((i["nagg"] * i["k"],), np.uint8),
                  12: ((i["nr"], i["b"], i["b"]), np.float64), 13: ((i["nr"] * i["b"], i["k"]), np.float64),
                  14: ((i["nr"] * i["b"], i["k"]), np.float64), 15: ((i["nr"],), np.uint8)}
        shape, dt = shapes[f]
        out = np.empty(shape, dt)
        if lib().orc_amg_level_get(self.h, l, f, _p(out)) != 0:
            return None
        return out

    def vcycle(self, b):
        b = _c(b, np.float64); x = np.empty_like(b)
        lib().orc_amg_vcycle(self.h, _p(b), _p(x))
        return x

    def smooth(self, l, b, x0=None):
        b = _c(b, np.float64)
        x = np.zeros_like(b) if x0 is None else _c(x0, np.float64).copy()
        lib().orc_amg_smooth(self.h, l, _p(b), _p(x), 1 if x0 is None else 0)
        return x


class Amg(Hierarchy):
    def __init__(self, rp, ci, val, B, opts=None):
        rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64)
        B = _c(B, np.float64)
        b = val.shape[1] if val.ndim == 3 else 1
        k = B.shape[1] if B.ndim == 2 else 1
        h = P()
        rc = lib().orc_amg_create(rp.size - 1, b, _p(rp), _p(ci), _p(val), _p(B), k,
                                  C.byref(opts or amg_opts()), C.byref(h))
        if rc:
            raise RuntimeError("oracle AMG setup failed")
        super().__init__(h, None)

    def update(self, val, B=None):
        """Numeric re-setup for new values on the same pattern (aggregates kept); B optional."""
        val = _c(val, np.float64)
        B = None if B is None else _c(B, np.float64)
        if lib().orc_amg_update(self.h, _p(val), None if B is None else _p(B)):
            raise RuntimeError("oracle AMG update failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_amg_free(self.h)
            self.h = None


class Scr:
    """Oracle SCR system built from the 4x4 BSR K (interleaved [vx vy vz p] per node)."""

    def __init__(self, rp, ci, val, xyz, opts=None):
        self.rp = _c(rp, np.int32); self.ci = _c(ci, np.int32); self.val = _c(val, np.float64)
        xyz = _c(xyz, np.float64)
        self.nb = self.rp.size - 1
        self.h = P()
        rc = lib().orc_scr_create(self.nb, _p(self.rp), _p(self.ci), _p(self.val), _p(xyz),
                                  C.byref(opts or amg_opts()), C.byref(self.h))
        if rc:
            raise RuntimeError("oracle SCR setup failed")
        self.amgA = Hierarchy(lib().orc_scr_amg(self.h, 0), self)
        self.amgS = Hierarchy(lib().orc_scr_amg(self.h, 1), self)

    def update(self, val, xyz=None):
        """Numeric re-setup for new values on the same pattern (aggregates kept)."""
        self.val = _c(val, np.float64)
        xyz = None if xyz is None else _c(xyz, np.float64)
        rc = lib().orc_scr_update(self.h, _p(self.val), None if xyz is None else _p(xyz))
        if rc:
            raise RuntimeError(f"oracle SCR update failed ({rc})")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scr_free(self.h)
            self.h = None

    def set_outlets(self, outlets, m):
        """Outlet resistance coupling: outlets = [(block rows, a (n, 3)), ...], m = coefficients;
        the solves' K and A gain sum_k m_k a_k a_k^T on the velocity dofs (empty list removes it)."""
        n = len(outlets)
        off = np.zeros(n + 1, np.int64)
        for k, (blk, a) in enumerate(outlets):
            off[k + 1] = off[k] + len(blk)
        blk = np.ascontiguousarray(np.concatenate([b for b, _ in outlets]) if n else np.zeros(1), np.int32)
        a = np.ascontiguousarray(np.concatenate([a for _, a in outlets]) if n else np.zeros((1, 3)), np.float64)
        mm = np.ascontiguousarray(m if n else np.zeros(1), np.float64)
        self._outlets = (off, blk, a, mm)
        if lib().orc_scr_set_outlets(self.h, n, _p(off), _p(blk), _p(a), _p(mm)):
            raise ValueError("invalid outlet data")

    def matrix(self, which):
        """which: 'A', 'G', 'D', 'C', 'Shat' -> (rp, ci, val)"""
        w = {"A": 0, "G": 1, "D": 2, "C": 3, "Shat": 4}[which]
        info = np.zeros(4, np.int64)
        lib().orc_scr_matrix(self.h, w, -1, _p(info))
        nr, nnz, br, bc = (int(v) for v in info)
        rp = np.empty(nr + 1, np.int32); ci = np.empty(nnz, np.int32); v = np.empty((nnz, br, bc))
        lib().orc_scr_matrix(self.h, w, 0, _p(rp))
        lib().orc_scr_matrix(self.h, w, 1, _p(ci))
        lib().orc_scr_matrix(self.h, w, 2, _p(v))
        return rp, ci, v

    def solve(self, b, opts=None, x0=None):
        b = _c(b, np.float64)
        o = opts or solve_opts()
        x = np.zeros_like(b) if x0 is None else _c(x0, np.float64).copy()
        if x0 is not None:
            o.use_x0 = 1
        st = ScrStats()
        rc = lib().orc_scr_solve(self.h, _p(b), _p(x), C.byref(o), C.byref(st))
        return x, rc, st.as_dict()

    OPS = {"K": (4, 4), "A": (3, 3), "VA": (3, 3), "VS": (1, 1), "S": (1, 1), "SCR": (4, 4),
           "G": (1, 3), "D": (3, 1), "C": (1, 1), "Shat": (1, 1), "SIMPLE": (4, 4), "d": (3, 3)}

    def apply(self, op, x, opts=None):
        """Split-layout component operators: see orc_scr_apply."""
        code = {"K": 0, "A": 1, "VA": 2, "VS": 3, "S": 4, "SCR": 5, "G": 6, "D": 7, "C": 8, "Shat": 9,
                "SIMPLE": 10, "d": 11}[op]
        nin, nout = self.OPS[op]
        x = _c(x, np.float64)
        assert x.size == nin * self.nb
        y = np.empty(nout * self.nb)
        lib().orc_scr_apply(self.h, code, _p(x), _p(y), C.byref(opts or solve_opts()))
        return y


class Mesh:
    def __init__(self, rp, ci, val, opts=None):
        self.rp = _c(rp, np.int32); self.ci = _c(ci, np.int32); self.val = _c(val, np.float64)
        self.n = self.rp.size - 1
        self.h = P()
        rc = lib().orc_mesh_create(self.n, _p(self.rp), _p(self.ci), _p(self.val),
                                   C.byref(opts or amg_opts()), C.byref(self.h))
        if rc:
            raise RuntimeError("oracle mesh setup failed")
        self.amg = Hierarchy(lib().orc_mesh_amg(self.h), self)

    def update(self, val):
        """Numeric re-setup for new Laplacian values on the same pattern (aggregates kept)."""
        self.val = _c(val, np.float64)
        if lib().orc_mesh_update(self.h, _p(self.val)):
            raise RuntimeError("oracle mesh update failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mesh_free(self.h)
            self.h = None

    def solve(self, b, tol=1e-8, maxit=500, flexible=False):
        b = _c(b, np.float64)
        x = np.empty_like(b)
        its = np.zeros(3, np.int64); rel = np.zeros(3)
        rc = lib().orc_mesh_solve(self.h, _p(b), _p(x), tol, maxit, int(flexible), _p(its), _p(rel))
        return x, rc, its, rel


def gmres(rp, ci, val, rhs, amg=None, tol=1e-10, maxit=500, restart=30):
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64); rhs = _c(rhs, np.float64)
    b = val.shape[1] if val.ndim == 3 else 1
    x = np.empty_like(rhs); its = np.zeros(1, np.int64); rel = np.zeros(1)
    rc = lib().orc_gmres(rp.size - 1, b, _p(rp), _p(ci), _p(val), amg.h if amg else None, _p(rhs), _p(x),
                         tol, maxit, restart, _p(its), _p(rel))
    return x, rc, int(its[0]), float(rel[0])


def cg(rp, ci, val, rhs, amg=None, tol=1e-10, maxit=500, flexible=False):
    rp = _c(rp, np.int32); ci = _c(ci, np.int32); val = _c(val, np.float64); rhs = _c(rhs, np.float64)
    x = np.empty_like(rhs); its = np.zeros(1, np.int64); rel = np.zeros(1)
    rc = lib().orc_cg(rp.size - 1, _p(rp), _p(ci), _p(val), amg.h if amg else None, _p(rhs), _p(x),
                      tol, maxit, int(flexible), _p(its), _p(rel))
    return x, rc, int(its[0]), float(rel[0])
