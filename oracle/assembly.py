"""FP64 CPU oracle of the corrector tangent assembly -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this module; the GPU library never calls it and shares no code with it.

What it computes (the fully discrete tangent of the corrector system of Sec. 3.5, divided by
alpha_f gamma dt, on P1 tetrahedra with every element integral taken by the one-point centroid
rule):

* generalized-alpha constants of the first-order system (Sec. 3.4): alpha_m = (3 - rho_inf) /
  (2 (1 + rho_inf)), alpha_f = 1 / (1 + rho_inf), gamma = 1/2 + alpha_m - alpha_f, and
  c_t = alpha_m / (alpha_f gamma dt), the factor that the time derivative contributes once the
  tangent is divided by alpha_f gamma dt;
* the fluid (Sec. 3.2, residual-based VMS): the Galerkin mass and viscous terms, the grad-div
  term weighted by tau_C, the pressure gradient / divergence pair, the pressure stabilisation
  tau_M grad q . grad p and, about an advective velocity u (Oseen form), the Galerkin convection,
  the reaction rho (grad u), and the fine-scale velocity v' = -tau_M r_M terms carried by
  ub . grad w (momentum), grad q (continuity) and grad p; tau_M and tau_C from the element
  metric G = J^-T M J^-1 with the regular-simplex matrix M;
* the solid (Sec. 3.1 with c_m = c_c = 0): mass, the deviatoric elastic stiffness scaled by
  alpha_f gamma dt / alpha_m (displacement increments are that multiple of velocity increments),
  and the pressure mass (c_t / kappa);
* assembly into the given 4x4 block pattern, with the velocity rows of a vertex at ``tv`` and
  its pressure row at ``tp`` (they differ on the fluid/solid interface, Sec. 3.3), then the
  symmetric elimination of Dirichlet dofs (rows and columns zeroed, unit diagonal).

The same routine also yields the three parts of the linear(ised) semi-discrete residual that the
predictor multi-corrector of Sec. 3.5 evaluates at the intermediate states, with no advection
(``form``): "rate" acts on the rates (v_dot, p_dot): rho M in both media, the fine-scale rate term
of the continuity row when it is enabled, and the solid pressure mass M / kappa; "state" acts on
(v, p): the fluid viscous and grad-div terms, the pressure gradient / divergence pair and the
fluid pressure stabilisation; "disp" acts on the solid displacement: the deviatoric elastic
stiffness with the plain modulus mu_s.  Their Dirichlet rows and columns are zero (no unit
diagonal).  Differentiating the residual at the intermediate states with respect to the velocity
rate, with the solid displacement rate tied to it by the kinematic equation, gives
tangent = c_t rate + state + disp / c_t.

Pinned in ``tests/test_assembly_oracle.py`` by patch tests on a uniform box (linear fields),
lumped-mass and lumped-volume identities, D = -G^T at rest, and agreement with the independently
written element integrals of the input generator (themselves pinned in ``tests/test_synth.py``);
the residual parts in ``tests/test_corrector_oracle.py`` (lumped masses, rigid motions, the
identity above at two step sizes, the medium each term lives in).
"""
from __future__ import annotations

import numpy as np

MASS, VISC, GRADDIV, GD, CPP, CONV = 1, 2, 4, 8, 16, 32
FORMS = ("tangent", "rate", "state", "disp")


def genalpha(rho_inf: float):
    """(alpha_m, alpha_f, gamma) of first-order generalized-alpha (Sec. 3.4)."""
    am = (3.0 - rho_inf) / (2.0 * (1.0 + rho_inf))
    af = 1.0 / (1.0 + rho_inf)
    return am, af, 0.5 + am - af


def shape_gradients(X: np.ndarray):
    """X: (ne, 4, 3) vertex coordinates.  Returns (grad N (ne, 4, 3), volume (ne,)).  The Jacobian
    of the map from the reference tetrahedron has columns x_k - x_0; the rows of its inverse are
    grad N_1..3, and grad N_0 = -(grad N_1 + grad N_2 + grad N_3)."""
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))      # J[e, i, k] = x_{k+1,i} - x_{0,i}
    Jinv = np.linalg.inv(J)                                      # Jinv[e, k, i] = d xi_k / d x_i
    dN = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    return dN, np.abs(np.linalg.det(J)) / 6.0


def stabilisation(dN: np.ndarray, ub: np.ndarray, rho: float, mu: float, dt: float):
    """tau_M, tau_C (Sec. 3.2) per element: G = J^-T M J^-1 with M = 2^(1/3)/2 [2 1 1; 1 2 1; 1 1 2],
    tau_M = (rho sqrt(C_T/dt^2 + ub.G.ub + C_I nu^2 G:G))^-1, C_T = 4, C_I = 36, nu = mu/rho,
    tau_C = (tau_M tr G)^-1."""
    M = (2.0 ** (1.0 / 3.0) / 2.0) * np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]])
    Jinv = dN[:, 1:, :]
    G = np.einsum("eki,kl,elj->eij", Jinv, M, Jinv)
    nu = mu / rho
    uGu = np.einsum("ei,eij,ej->e", ub, G, ub)
    tauM = 1.0 / (rho * np.sqrt(4.0 / dt ** 2 + uGu + 36.0 * nu ** 2 * np.einsum("eij,eij->e", G, G)))
    tauC = 1.0 / (tauM * np.trace(G, axis1=1, axis2=2))
    return tauM, tauC


def _coefficients(form: str, ct: float, mu_f: float, visc_s: float, mu_s: float, kappa: float):
    """Weight of each term in one assembled form: (mass, fluid viscosity, solid elastic modulus,
    grad-div, G/D pair, fine-scale rate term, fluid pressure stabilisation, solid pressure mass)."""
    if form == "tangent":
        return dict(mass=ct, visc_f=mu_f, visc_s=visc_s, graddiv=1.0, gd=1.0, dtc=ct, cpp_f=1.0, cpp_s=ct / kappa)
    if form == "rate":
        return dict(mass=1.0, visc_f=0.0, visc_s=0.0, graddiv=0.0, gd=0.0, dtc=1.0, cpp_f=0.0, cpp_s=1.0 / kappa)
    if form == "state":
        return dict(mass=0.0, visc_f=mu_f, visc_s=0.0, graddiv=1.0, gd=1.0, dtc=0.0, cpp_f=1.0, cpp_s=0.0)
    if form == "disp":
        return dict(mass=0.0, visc_f=0.0, visc_s=mu_s, graddiv=0.0, gd=0.0, dtc=0.0, cpp_f=0.0, cpp_s=0.0)
    raise ValueError(f"unknown form {form!r}")


def element_matrices(X, solid, U, prm: dict, form: str = "tangent") -> np.ndarray:
    """Element tangents Ke[e, a, i, b, j] (i, j = 0..2 velocity, 3 pressure) of Sec. 3.5 divided by
    alpha_f gamma dt, or one residual part (``form``, see the module docstring; advection only in
    the tangent).  X: (ne, 4, 3); solid: (ne,) bool; U: (ne, 4, 3) advective velocity at the
    vertices or None (at rest); prm: rho_f, mu_f, rho_s, E_s, nu_s, dt, rho_inf, terms,
    vms_dt_coupling."""
    ne = X.shape[0]
    terms = int(prm["terms"])
    am, af, gam = genalpha(prm["rho_inf"])
    dt = prm["dt"]
    ct = am / (af * gam * dt)
    mu_s = prm["E_s"] / (2.0 * (1.0 + prm["nu_s"]))
    kappa = prm["E_s"] / (3.0 * (1.0 - 2.0 * prm["nu_s"]))
    w = _coefficients(form, ct, prm["mu_f"], (af * gam * dt / am) * mu_s, mu_s, kappa)
    dN, V = shape_gradients(X)
    fluid = ~solid
    conv = (terms & CONV) != 0 and U is not None and form == "tangent"
    ub = np.zeros((ne, 3))
    gu = np.zeros((ne, 3, 3))                                    # gu[e, i, j] = d u_i / d x_j
    if conv:
        ub = np.where(fluid[:, None], U.mean(axis=1), 0.0)
        gu = np.where(fluid[:, None, None], np.einsum("eai,eaj->eij", U, dN), 0.0)
    tauM, tauC = stabilisation(dN, ub, prm["rho_f"], prm["mu_f"], dt)
    tauM = np.where(fluid, tauM, 0.0)
    tauC = np.where(fluid, tauC, 0.0)
    rho = np.where(fluid, prm["rho_f"], prm["rho_s"])
    visc = np.where(fluid, w["visc_f"], w["visc_s"])

    I3 = np.eye(3)
    Mab = V[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0           # P1 mass matrix
    Lab = V[:, None, None] * np.einsum("eai,ebi->eab", dN, dN)                     # P1 stiffness
    ua = np.einsum("ei,eai->ea", ub, dN)                                           # ub . grad N_a
    Ke = np.zeros((ne, 4, 4, 4, 4))
    Avv = np.zeros((ne, 4, 3, 4, 3))
    if terms & MASS:
        Avv += (rho * w["mass"])[:, None, None, None, None] * np.einsum("eab,ij->eaibj", Mab, I3)
    if terms & VISC:
        Avv += visc[:, None, None, None, None] * (
            np.einsum("eab,ij->eaibj", Lab, I3)
            + V[:, None, None, None, None] * np.einsum("eaj,ebi->eaibj", dN, dN)
            - (2.0 / 3.0) * V[:, None, None, None, None] * np.einsum("eai,ebj->eaibj", dN, dN))
    if terms & GRADDIV:
        Avv += (w["graddiv"] * tauC * V)[:, None, None, None, None] * np.einsum("eai,ebj->eaibj", dN, dN)
    if conv:
        # Galerkin convection rho w . (ub . grad) v and reaction rho w . (grad u) v
        # (N_a at the centroid is 1/4 for every a)
        gal = (rho * V / 4.0)[:, None, None] * np.broadcast_to(ua[:, None, :], (ne, 4, 4))
        Avv += np.einsum("eab,ij->eaibj", gal, I3)
        Avv += rho[:, None, None, None, None] * np.einsum("eab,eij->eaibj", Mab, gu)
        # fine scales: (ub . grad w) . tau_M rho (rho c_t v + rho (ub . grad) v), at the centroid
        supg = (tauM * rho * rho)[:, None, None] * ua[:, :, None] * (
            ct * (V / 4.0)[:, None, None] + V[:, None, None] * ua[:, None, :])
        Avv += np.einsum("eab,ij->eaibj", supg, I3)
    Ke[:, :, :3, :, :3] = Avv
    if terms & GD:
        # -(p, div w) and (q, div v) with p, v at the centroid: V/4 per vertex value
        Ke[:, :, :3, :, 3] = -(w["gd"] * V / 4.0)[:, None, None, None] * dN[:, :, :, None]
        Ke[:, :, 3, :, :3] = (w["gd"] * V / 4.0)[:, None, None, None] * dN[:, None, :, :]
        if prm.get("vms_dt_coupling", 0):
            Ke[:, :, 3, :, :3] += (w["dtc"] * rho * tauM * V / 4.0)[:, None, None, None] * dN[:, :, None, :]
    if conv:
        # grad p through v' in the momentum row: (ub . grad w) tau_M rho grad p
        Ke[:, :, :3, :, 3] += (tauM * rho * V)[:, None, None, None] * ua[:, :, None, None] * \
            np.transpose(dN, (0, 2, 1))[:, None, :, :]
        # (grad q) . tau_M rho (ub . grad) v in the continuity row
        Ke[:, :, 3, :, :3] += (tauM * rho * V)[:, None, None, None] * dN[:, :, None, :] * ua[:, None, :, None]
    if terms & CPP:
        Ke[:, :, 3, :, 3] = np.where(fluid[:, None, None], w["cpp_f"] * tauM[:, None, None] * Lab,
                                     w["cpp_s"] * Mab)
    return Ke


def _positions(rp, ci, rows, cols):
    """Index of block (rows[k], cols[k]) in the pattern (rows sorted by column)."""
    nb = rp.size - 1
    key = np.repeat(np.arange(nb, dtype=np.int64), np.diff(rp)) * nb + ci
    want = rows.astype(np.int64) * nb + cols
    q = np.searchsorted(key, want)
    if np.any(q >= key.size) or np.any(key[np.minimum(q, key.size - 1)] != want):
        raise ValueError("an element couples two block rows the pattern does not hold")
    return q


def tangent(tv, tp, tsolid, xyz, rp, ci, mask, prm: dict, u=None, rows=None, chunk: int = 100_000,
            form: str = "tangent"):
    """Assembled tangent values (nnzb, 4, 4) on the pattern (rp, ci), Dirichlet dofs (mask, 4 per
    block row) eliminated.  u: (n_b, 3) advective velocity or None.  rows: optional block rows;
    then only the elements touching them are assembled and only those rows are exact.  form: one
    of FORMS; the residual parts keep zero Dirichlet rows and columns."""
    tv = np.asarray(tv); tp = np.asarray(tp)
    solid = np.asarray(tsolid).astype(bool)
    nb = rp.size - 1
    val = np.zeros((ci.size, 4, 4))
    elems = np.arange(tv.shape[0])
    if rows is not None:
        sel = np.zeros(nb, bool)
        sel[np.asarray(rows)] = True
        elems = elems[np.any(sel[tv] | sel[tp], axis=1)]
    for s in range(0, elems.size, chunk):
        e = elems[s:s + chunk]
        X = xyz[tv[e]]
        U = None if u is None else u[tv[e]]
        Ke = element_matrices(X, solid[e], U, prm, form)
        for a in range(4):
            for b in range(4):
                q = _positions(rp, ci, tv[e, a], tv[e, b])
                np.add.at(val, (q, slice(0, 3), slice(0, 3)), Ke[:, a, :3, b, :3])
                q = _positions(rp, ci, tv[e, a], tp[e, b])
                np.add.at(val, (q, slice(0, 3), 3), Ke[:, a, :3, b, 3])
                q = _positions(rp, ci, tp[e, a], tv[e, b])
                np.add.at(val, (q, 3, slice(0, 3)), Ke[:, a, 3, b, :3])
                q = _positions(rp, ci, tp[e, a], tp[e, b])
                np.add.at(val, (q, 3, 3), Ke[:, a, 3, b, 3])
    # symmetric elimination of the Dirichlet dofs
    m = np.asarray(mask).reshape(nb, 4).astype(bool)
    rowof = np.repeat(np.arange(nb), np.diff(rp))
    kill = m[rowof][:, :, None] | m[ci][:, None, :]
    val[kill] = 0.0
    if form != "tangent":
        return val
    diag = np.nonzero(rowof == ci)[0]
    for i in range(4):
        d = diag[m[rowof[diag], i]]
        val[d, i, i] = 1.0
    return val


def params_of(p) -> dict:
    """The physical constants of a generator parameter set as a dict."""
    return {k: getattr(p, k) for k in ("rho_f", "mu_f", "rho_s", "E_s", "nu_s", "dt", "rho_inf", "terms",
                                         "vms_dt_coupling")}
