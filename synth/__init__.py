"""Seeded synthetic inputs: tube meshes, the 4x4-block tangent K, the mesh-motion Laplacian L
and right-hand sides.

This module is the only code shared by the oracle side and the GPU side, and it holds none of
the solver's arithmetic: it produces the linear systems the paper's Section 3.5 states
(the 2x2 velocity/pressure corrector system and the mesh-motion system), nothing else.
The C source is ``synth/synth.c``; :func:`build` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    src = os.path.join(_HERE, "synth.c")
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
           src, "-o", _SO + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [("mode", C.c_int), ("m_core", C.c_int), ("n_bl", C.c_int), ("n_wall", C.c_int),
                ("nz", C.c_int), ("R", C.c_double), ("L", C.c_double), ("wall_ratio", C.c_double),
                ("bl_ratio", C.c_double), ("rho_f", C.c_double), ("mu_f", C.c_double),
                ("rho_s", C.c_double), ("E_s", C.c_double), ("nu_s", C.c_double), ("dt", C.c_double),
                ("rho_inf", C.c_double), ("terms", C.c_int), ("apply_bc", C.c_int),
                ("vms_dt_coupling", C.c_int), ("box_solid", C.c_int), ("y_h", C.c_double),
                ("y_rd", C.c_double), ("y_ld", C.c_double), ("y_th1", C.c_double), ("y_th2", C.c_double),
                ("u_max", C.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = C.CDLL(_SO)
        P = C.c_void_p
        lib.synth_build.argtypes = [C.POINTER(Params), C.POINTER(P)]
        lib.synth_build.restype = C.c_int
        lib.synth_info.argtypes = [P, P]
        lib.synth_get_K.argtypes = [P, P, P, P]
        lib.synth_get_nodes.argtypes = [P, P, P, P]
        lib.synth_get_L.argtypes = [P, P, P, P, P, P]
        lib.synth_get_tets.argtypes = [P, P, P, P, P]
        lib.synth_get_flow.argtypes = [P, P, P, P, P]
        lib.synth_free.argtypes = [P]
        lib.synth_rhs.argtypes = [C.c_uint64, C.c_int64, P, P]
        lib.synth_element.argtypes = [P, P, C.POINTER(Params), C.c_int, P]
        lib.synth_element.restype = C.c_double
        lib.synth_tau.argtypes = [P, P, C.POINTER(Params), P, P]
        lib.synth_genalpha.argtypes = [C.c_double, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_params(**kw) -> Params:
    """Physical constants of the fluid/solid workloads: rho=1.06, mu=0.04, dt=1e-3,
    rho_inf=0.5; solid E=1e6, nu=0.45, rho_s=1.0 (cgs units as in the paper's Section 6).
    At rest (u_max = 0) unless an advective centreline speed u_max is given."""
    p = Params(mode=0, m_core=6, n_bl=0, n_wall=0, nz=40, R=1.0, L=5.0, wall_ratio=1.2,
               bl_ratio=0.6, rho_f=1.06, mu_f=0.04, rho_s=1.0, E_s=1.0e6, nu_s=0.45, dt=1.0e-3,
               rho_inf=0.5, terms=63, apply_bc=1, vms_dt_coupling=0, box_solid=0, y_h=0.0, y_rd=0.7,
               y_ld=5.0, y_th1=0.0, y_th2=0.0, u_max=0.0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class System(dict):
    """Attribute-style access to the arrays of one generated system."""

    def __getattr__(self, k):
        try:
            return self[k]
        except KeyError as e:
            raise AttributeError(k) from e


def generate(p: Params, tets: bool = False) -> System:
    lib = _load()
    h = C.c_void_p()
    rc = lib.synth_build(C.byref(p), C.byref(h))
    if rc != 0:
        raise RuntimeError(f"synth_build failed ({rc})")
    try:
        info = np.zeros(10, np.int64)
        lib.synth_info(h, _ptr(info))
        n_phys, nb, nnzb, nt, nnzL, nif, S, nzn, n_out, n_oe = (int(v) for v in info)
        rp = np.empty(nb + 1, np.int32); ci = np.empty(nnzb, np.int32)
        val = np.empty((nnzb, 4, 4), np.float64)
        lib.synth_get_K(h, _ptr(rp), _ptr(ci), _ptr(val))
        xyz = np.empty((nb, 3)); mask = np.empty(4 * nb, np.uint8); kind = np.empty(nb, np.uint8)
        lib.synth_get_nodes(h, _ptr(xyz), _ptr(mask), _ptr(kind))
        Lrp = np.empty(n_phys + 1, np.int32); Lci = np.empty(nnzL, np.int32)
        Lval = np.empty(nnzL); Lmask = np.empty(n_phys, np.uint8); Lxyz = np.empty((n_phys, 3))
        lib.synth_get_L(h, _ptr(Lrp), _ptr(Lci), _ptr(Lval), _ptr(Lmask), _ptr(Lxyz))
        uadv = np.empty((nb, 3)); ooff = np.empty(n_out + 1, np.int64)
        oblk = np.empty(max(n_oe, 1), np.int32); oa = np.empty((max(n_oe, 1), 3))
        lib.synth_get_flow(h, _ptr(uadv), _ptr(ooff), _ptr(oblk), _ptr(oa))
        outlets = [(oblk[ooff[k]:ooff[k + 1]].copy(), oa[ooff[k]:ooff[k + 1]].copy()) for k in range(n_out)]
        out = System(n_phys=n_phys, n_b=nb, nnzb=nnzb, n_tets=nt, n_iface=nif, section=S,
                     layers=nzn, rp=rp, ci=ci, val=val, xyz=xyz, mask=mask, kind=kind,
                     Lrp=Lrp, Lci=Lci, Lval=Lval, Lmask=Lmask, Lxyz=Lxyz, uadv=uadv, outlets=outlets)
        if tets:
            tv = np.empty((nt, 4), np.int32); tp = np.empty((nt, 4), np.int32)
            ts = np.empty(nt, np.uint8); bop = np.empty(n_phys, np.int32)
            lib.synth_get_tets(h, _ptr(tv), _ptr(tp), _ptr(ts), _ptr(bop))
            out.update(tv=tv, tp=tp, tsolid=ts, blk_of_phys=bop)
        return out
    finally:
        lib.synth_free(h)


def rhs(seed: int, n: int, mask: np.ndarray | None = None) -> np.ndarray:
    """Uniform[-1,1) per entry from splitmix64, zero where mask != 0."""
    lib = _load()
    out = np.empty(n)
    m = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    lib.synth_rhs(C.c_uint64(seed & (2**64 - 1)), n, None if m is None else _ptr(m), _ptr(out))
    return out


def element(x4: np.ndarray, p: Params, solid: bool = False, u4: np.ndarray | None = None):
    """16x16 element matrix (index 4*a + c) of one tetrahedron; u4: advective velocity at its
    4 vertices (4x3) or None (at rest)."""
    lib = _load()
    x = np.ascontiguousarray(x4, np.float64).reshape(12)
    u = None if u4 is None else np.ascontiguousarray(u4, np.float64).reshape(12)
    Ke = np.empty((16, 16))
    V = lib.synth_element(_ptr(x), None if u is None else _ptr(u), C.byref(p), int(solid), _ptr(Ke))
    return Ke, V


def tau(x4: np.ndarray, p: Params, ub: np.ndarray | None = None):
    lib = _load()
    x = np.ascontiguousarray(x4, np.float64).reshape(12)
    u = None if ub is None else np.ascontiguousarray(ub, np.float64).reshape(3)
    a = np.zeros(1); b = np.zeros(1)
    lib.synth_tau(_ptr(x), None if u is None else _ptr(u), C.byref(p), _ptr(a), _ptr(b))
    return float(a[0]), float(b[0])


def genalpha(rho_inf: float):
    lib = _load()
    a, b, c = np.zeros(1), np.zeros(1), np.zeros(1)
    lib.synth_genalpha(rho_inf, _ptr(a), _ptr(b), _ptr(c))
    return float(a[0]), float(b[0]), float(c[0])


# ---------------------------------------------------------------- workload presets
def cfg0_params() -> Params:
    """Straight fluid tube R=1, L=5, 12x12x40 cells (6,929 nodes)."""
    return default_params(mode=0, m_core=6, n_bl=0, n_wall=0, nz=40, R=1.0, L=5.0)


def cfg1_params() -> Params:
    """Unified fluid+solid tube: lumen R=1 (12 core + 4 boundary-layer shells, factor 0.6),
    wall 1.0-1.2 (4 shells), L=10, 178 axial cells: 41x41x179 = 300,899 nodes."""
    return default_params(mode=0, m_core=12, n_bl=4, n_wall=4, nz=178, R=1.0, L=10.0)


def cfg2_params() -> Params:
    """cfg1 refined: 24 core + 4 BL + 6 wall shells, 305 axial cells: 69x69x306 nodes."""
    return default_params(mode=0, m_core=24, n_bl=4, n_wall=6, nz=305, R=1.0, L=10.0)


def tube_params(n_nodes: float, R: float, L: float) -> Params:
    """A unified tube with about n_nodes nodes, lumen radius R, length L (serving requests):
    core/BL/wall shells in the cfg1 proportions (3:1:1), axial spacing ~ core spacing."""
    best = None
    for m_core in range(3, 80):
        n_bl, n_wall = 4, max(2, round(m_core / 3))
        m = m_core + n_bl + n_wall
        S = 1.0 + sum(0.6 ** t for t in range(n_bl))
        hc = (R / (1.0 + S / m_core)) / m_core
        nz = max(4, round(L / hc))
        n = (2 * m + 1) ** 2 * (nz + 1)
        if best is None or abs(math.log(n / n_nodes)) < abs(math.log(best[0] / n_nodes)):
            best = (n, m_core, n_bl, n_wall, nz)
    _, m_core, n_bl, n_wall, nz = best
    return default_params(mode=0, m_core=m_core, n_bl=n_bl, n_wall=n_wall, nz=nz, R=R, L=L)


def y_params(n_nodes: float | None = None, seed: int = 0, h: float | None = None, Lp: float = 5.0,
             Ld: float = 5.0) -> Params:
    """Y-bifurcation on a voxel grid: parent radius 1 and length Lp along +z up to the junction,
    daughters of radius 0.7 and length Ld at seeded angles U[30, 60] degrees from the z axis in
    the x-z plane (one toward +x, one toward -x), wall out to 1.2x the local radius.  The voxel
    spacing is h, or chosen so that the mesh has about n_nodes nodes."""
    rng = np.random.default_rng(seed)
    th1, th2 = np.deg2rad(rng.uniform(30.0, 60.0, 2))
    if h is None:
        W, rd = 1.2, 0.7
        vol = math.pi * W ** 2 * Lp + 2 * math.pi * (W * rd) ** 2 * Ld + 4.0 / 3.0 * math.pi * W ** 3 / 2
        vol *= 0.935     # the branches overlap at the junction (measured: 3.74M nodes for 4.0M unscaled)
        h = (vol / n_nodes) ** (1.0 / 3.0)
    return default_params(mode=2, R=1.0, L=Lp, wall_ratio=1.2, y_h=h, y_rd=0.7, y_ld=Ld, y_th1=float(th1),
                          y_th2=float(th2))


def cfg4_params() -> Params:
    """Largest single-GPU workload: the Y-bifurcation with about 4.0M nodes (angle seed 0)."""
    return y_params(4.0e6, seed=0)


def tiny_annulus_params() -> Params:
    """5x5 section (1 core + 1 wall shell), 3 axial cells: the smallest fluid+solid system."""
    return default_params(mode=0, m_core=1, n_bl=0, n_wall=1, nz=3, R=1.0, L=1.0)
