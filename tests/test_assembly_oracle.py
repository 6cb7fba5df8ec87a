"""Pins of the tangent-assembly oracle (oracle/assembly.py) against facts that do not come from
it: patch tests on a uniform box (P1 reproduces linear fields, so interior rows of the
linearised operators act on them exactly as the continuous operators do), lumped-mass and
lumped-volume identities, D = -G^T at rest, a closed form of the convection and fine-scale
momentum terms for an advective velocity along the Kuhn diagonal, and agreement with the input
generator's independently written element integrals (pinned in test_synth.py)."""
import numpy as np
import pytest

import synth
from oracle import assembly as asm

H = 0.5


def box(**kw):
    p = synth.default_params(mode=1, m_core=6, n_bl=5, nz=5, R=H, apply_bc=0, **kw)
    return p, synth.generate(p, tets=True)


def assemble(p, s, u=None, **over):
    prm = asm.params_of(p)
    prm.update(over)
    return asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, prm, u=u)


def apply(s, val, x):
    """y = K x for block values val (nnzb, 4, 4), x (n_b, 4)."""
    rowof = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    y = np.zeros((s.n_b, 4))
    np.add.at(y, rowof, np.einsum("qij,qj->qi", val, x[s.ci]))
    return y


def interior(s):
    lo, hi = s.xyz.min(0), s.xyz.max(0)
    return np.all((s.xyz > lo + 1e-9) & (s.xyz < hi - 1e-9), axis=1)


@pytest.mark.parametrize("kw", [
    dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=6, R=1.0, L=2.0),
    dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=6, R=1.0, L=2.0, u_max=30.0),
    dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=6, R=1.0, L=2.0, u_max=30.0, vms_dt_coupling=1, apply_bc=0),
    dict(mode=1, m_core=4, n_bl=3, nz=3, R=0.5, box_solid=1, apply_bc=0),
    dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=4, R=1.0, L=2.0, terms=8 | 16),
])
def test_matches_the_generators_element_integrals(kw):
    p = synth.default_params(**kw)
    s = synth.generate(p, tets=True)
    v = assemble(p, s, u=s.uadv if p.u_max else None)
    rowof = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    rmax = np.zeros(s.n_b)
    np.maximum.at(rmax, rowof, np.abs(s.val).reshape(-1, 16).max(1))
    assert np.all(np.abs(v - s.val).reshape(-1, 16).max(1) <= 1e-13 * rmax[rowof])


@pytest.mark.parametrize("solid", [0, 1])
def test_viscous_and_graddiv_terms_annihilate_linear_fields_at_interior_nodes(solid):
    p, s = box(box_solid=solid, terms=asm.VISC | asm.GRADDIV)
    v = assemble(p, s)
    B = np.random.default_rng(1).normal(size=(3, 3))
    x = np.zeros((s.n_b, 4))
    x[:, :3] = s.xyz @ B.T
    y = apply(s, v, x)
    inn = interior(s)
    assert inn.sum() > 20
    scale = np.abs(v).max() * np.abs(x).max()
    assert np.abs(y[inn]).max() <= 1e-12 * scale
    assert np.abs(y[~inn]).max() > 1e-3 * scale          # not trivially zero


def test_mass_rows_sum_to_the_lumped_nodal_volume():
    p, s = box(terms=asm.MASS)
    v = assemble(p, s)
    am, af, g = asm.genalpha(p.rho_inf)
    ct = am / (af * g * p.dt)
    vol = np.prod(s.xyz.max(0) - s.xyz.min(0))
    for k in range(3):
        x = np.zeros((s.n_b, 4)); x[:, k] = 1.0
        y = apply(s, v, x)
        assert np.allclose(y[interior(s), k], p.rho_f * ct * H ** 3, rtol=1e-13)
        assert np.isclose(y[:, k].sum(), p.rho_f * ct * vol, rtol=1e-12)
        assert np.abs(np.delete(y, k, axis=1)).max() == 0.0


def test_gradient_of_a_linear_pressure_and_D_is_minus_G_transpose():
    p, s = box(terms=asm.GD)
    v = assemble(p, s)
    gvec = np.array([0.3, -1.1, 0.7])
    x = np.zeros((s.n_b, 4)); x[:, 3] = s.xyz @ gvec + 2.0
    y = apply(s, v, x)
    inn = interior(s)
    # -(p, div w) = (grad p, w) for w vanishing on the patch boundary: g_i times the lumped volume
    assert np.allclose(y[inn, :3], gvec[None, :] * H ** 3, rtol=1e-12, atol=1e-15)
    rowof = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    Gd = np.zeros((s.n_b, 3, s.n_b)); Dd = np.zeros((s.n_b, s.n_b, 3))
    Gd[rowof, :, s.ci] = v[:, :3, 3]
    Dd[rowof, s.ci, :] = v[:, 3, :3]
    assert np.abs(Dd + np.transpose(Gd, (2, 0, 1))).max() == 0.0


def test_pressure_stabilisation_and_solid_pressure_mass():
    p, s = box(terms=asm.CPP)
    v = assemble(p, s)
    x = np.zeros((s.n_b, 4)); x[:, 3] = 1.0
    assert np.abs(apply(s, v, x)[:, 3]).max() <= 1e-14 * np.abs(v).max()
    x[:, 3] = s.xyz @ np.array([1.0, 2.0, -0.5])
    # tau_M is equal on every element of the uniform Kuhn box (congruent tetrahedra)
    assert np.abs(apply(s, v, x)[interior(s), 3]).max() <= 1e-12 * np.abs(v).max() * np.abs(x).max()
    p, s = box(terms=asm.CPP, box_solid=1)
    v = assemble(p, s)
    am, af, g = asm.genalpha(p.rho_inf)
    kappa = p.E_s / (3.0 * (1.0 - 2.0 * p.nu_s))
    x = np.zeros((s.n_b, 4)); x[:, 3] = 1.0
    y = apply(s, v, x)
    assert np.allclose(y[interior(s), 3], am / (af * g * p.dt) / kappa * H ** 3, rtol=1e-13)


def test_convection_along_the_kuhn_diagonal_closed_form():
    """Uniform u = s (1, 1, 1) on the box, mu = 0, only the convection terms (bit 32): grad u = 0,
    and on every Kuhn tetrahedron u.G.u = 2^(1/3) s^2 / h^2 (G = J^-T M J^-1 with J^-1 u =
    (0, 0, s/h)), so tau_M = 1 / (rho sqrt(4/dt^2 + 2^(1/3) s^2/h^2)) everywhere.  For w = B x, at
    an interior node a (integration by parts, div u = 0, the centroid rule exact on linear
    integrands, lumped volume h^3):
      Galerkin   sum_e rho V_e/4 (B u)                      = rho (B u) h^3
      fine scale sum_e tau rho^2 V_e (u.grad N_a)(c_t w(x_c) + B u) = -tau rho^2 c_t (B u) h^3."""
    sp = 7.0
    p, s = box(terms=asm.CONV, mu_f=0.0)
    u = np.full((s.n_b, 3), sp)
    v = assemble(p, s, u=u)
    B = np.random.default_rng(2).normal(size=(3, 3))
    x = np.zeros((s.n_b, 4)); x[:, :3] = s.xyz @ B.T
    y = apply(s, v, x)
    am, af, g = asm.genalpha(p.rho_inf)
    ct = am / (af * g * p.dt)
    rho = p.rho_f
    tau = 1.0 / (rho * np.sqrt(4.0 / p.dt ** 2 + 2.0 ** (1.0 / 3.0) * sp ** 2 / H ** 2))
    want = rho * (1.0 - tau * rho * ct) * (B @ u[0]) * H ** 3
    inn = interior(s)
    assert np.allclose(y[inn, :3], want[None, :], rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_dirichlet_elimination_and_interface_rows():
    p = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=4, R=1.0, L=2.0)
    s = synth.generate(p, tets=True)
    v = assemble(p, s)
    m = s.mask.reshape(-1, 4).astype(bool)
    rowof = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    for q in np.nonzero(rowof == s.ci)[0]:
        r = rowof[q]
        for i in range(4):
            if m[r, i]:
                assert v[q, i, i] == 1.0
                assert np.count_nonzero(v[rowof == r][:, i, :]) == 1
    # virtual (duplicated interface pressure) rows exist and carry only solid pressure coupling
    assert np.count_nonzero(s.kind == 3) > 0
    assert np.all(m[s.kind == 3, :3])


def test_rows_subset_matches_full_assembly():
    p = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=6, R=1.0, L=2.0, u_max=20.0)
    s = synth.generate(p, tets=True)
    full = assemble(p, s, u=s.uadv)
    rows = np.array([0, 5, s.n_b // 2, s.n_b - 1])
    part = asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, asm.params_of(p), u=s.uadv, rows=rows)
    for r in rows:
        sl = slice(s.rp[r], s.rp[r + 1])
        assert np.array_equal(part[sl], full[sl])


def test_generalized_alpha_constants_special_cases():
    # rho_inf = 1: no high-frequency damping, alpha_m = alpha_f = gamma = 1/2 (trapezoidal rule);
    # rho_inf = 0: alpha_m = 3/2, alpha_f = gamma = 1; in general gamma = 1/(1 + rho_inf) and the
    # scheme keeps second order (gamma = 1/2 + alpha_m - alpha_f)
    assert asm.genalpha(1.0) == (0.5, 0.5, 0.5)
    assert asm.genalpha(0.0) == (1.5, 1.0, 1.0)
    for r in (0.2, 0.5, 0.8):
        am, af, g = asm.genalpha(r)
        assert abs(g - 1.0 / (1.0 + r)) < 1e-15 and abs(af - 1.0 / (1.0 + r)) < 1e-15
        assert abs(am - (3.0 - r) / (2.0 * (1.0 + r))) < 1e-15
