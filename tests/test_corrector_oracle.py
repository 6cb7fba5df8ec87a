"""Pins of the time-integration oracle (oracle/corrector.py) and of the residual parts of the
assembly oracle (oracle/assembly.py, ``form``), against facts that do not come from the oracle:

* the residual parts: lumped masses and volumes computed from the vertex coordinates, the strain
  energy of linear displacement fields (2 mu V |dev sym A|^2), zero action on rigid motions, each
  term in its medium, and the linearisation identity tangent = c_t rate + state + disp / c_t at two
  step sizes;
* the time step: a monolithic solve of the generalized-alpha equations written from their
  definition (Sec. 3.4) on the small fluid/solid tube; the kinematic equation after the step; the
  scheme's relation between mesh displacement and mesh velocity;
* second-order convergence against the exact solutions of an oscillator (the solid's velocity
  form) and a decaying pressure mode; exact conservation of the oscillator's energy at
  rho_inf = 1 (the scheme is then the implicit midpoint rule);
* the harmonic extension reproducing constant Dirichlet data.
A planted mistake (a sign in the kinematic update) must fail the monolithic comparison.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import assembly as asm
from oracle import corrector as cor

SMALL = dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)


@pytest.fixture(scope="module")
def fsi():
    p = synth.default_params(**SMALL)
    return p, synth.generate(p, tets=True)


@pytest.fixture(scope="module")
def fsi_free():
    """the same tube with natural boundaries everywhere (no Dirichlet elimination)"""
    p = synth.default_params(apply_bc=0, **SMALL)
    return p, synth.generate(p, tets=True)


def _volumes(s):
    X = s.xyz[s.tv]
    e = X[:, 1:, :] - X[:, :1, :]
    return np.abs(np.linalg.det(e)) / 6.0


def _form(s, prm, form, dt=None):
    q = dict(prm)
    if dt is not None:
        q["dt"] = dt
    return cor.scalar_csr(s.rp, s.ci, asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, q, form=form))


def _field(nb, v=None, p=None):
    y = np.zeros((nb, 4))
    if v is not None:
        y[:, :3] = v
    if p is not None:
        y[:, 3] = p
    return y.reshape(-1)


# ------------------------------------------------------------------------- residual parts
@pytest.mark.parametrize("dtc", [0, 1])
def test_forms_combine_into_the_tangent(fsi, dtc):
    p, s = fsi
    prm = asm.params_of(p)
    prm["vms_dt_coupling"] = dtc
    am, af, g = asm.genalpha(prm["rho_inf"])
    m = s.mask.astype(bool)
    for dt in (1e-3, 3.7e-2):
        ct = am / (af * g * dt)
        K = {f: _form(s, prm, f, dt) for f in asm.FORMS}
        comb = ct * K["rate"] + K["state"] + K["disp"] / ct
        diff = (K["tangent"] - comb).toarray()
        # the only difference: the unit diagonal of the Dirichlet dofs
        expect = np.diag(m.astype(float))
        scale = abs(K["tangent"]).max()
        assert np.abs(diff - expect).max() <= 1e-13 * scale
        for f in ("rate", "state", "disp"):
            A = K[f].tocsr()
            assert abs(A[m]).max() == 0.0 and abs(A[:, m]).max() == 0.0


def test_rate_form_is_the_mass_of_both_media(fsi_free):
    p, s = fsi_free
    prm = asm.params_of(p)
    V = _volumes(s)
    sol = s.tsolid.astype(bool)
    Kr = _form(s, prm, "rate")
    nb = s.n_b
    ones = np.ones(nb)
    rho_vol = p.rho_f * V[~sol].sum() + p.rho_s * V[sol].sum()
    for c in range(3):
        e = np.zeros(3); e[c] = 1.0
        u = _field(nb, v=np.outer(ones, e))
        assert u @ (Kr @ u) == pytest.approx(rho_vol, rel=1e-13)
    # pressure: the solid pressure mass V / kappa (the fine-scale rate term is off); fluid rows none
    kappa = p.E_s / (3.0 * (1.0 - 2.0 * p.nu_s))
    q = _field(nb, p=ones)
    assert q @ (Kr @ q) == pytest.approx(V[sol].sum() / kappa, rel=1e-13)
    # no coupling of velocity and pressure in the rate form without the fine-scale rate term
    u = _field(nb, v=np.outer(ones, [1.0, 2.0, 3.0]))
    assert abs(q @ (Kr @ u)) <= 1e-12 * rho_vol


def _dev_sym_sq(A):
    S = 0.5 * (A + A.T)
    D = S - np.trace(S) / 3.0 * np.eye(3)
    return float((D * D).sum())


def test_disp_form_is_the_deviatoric_strain_energy_of_the_solid(fsi_free):
    p, s = fsi_free
    prm = asm.params_of(p)
    Kd = _form(s, prm, "disp")
    V = _volumes(s)
    sol = s.tsolid.astype(bool)
    mu_s = p.E_s / (2.0 * (1.0 + p.nu_s))
    rng = np.random.default_rng(3)
    for _ in range(3):
        A = rng.standard_normal((3, 3))
        u = _field(s.n_b, v=s.xyz @ A.T)
        assert u @ (Kd @ u) == pytest.approx(2.0 * mu_s * V[sol].sum() * _dev_sym_sq(A), rel=1e-11)
    # rigid motions: translations and infinitesimal rotations give zero force
    scale = abs(Kd).max()
    for c in range(3):
        e = np.zeros(3); e[c] = 1.0
        assert np.abs(Kd @ _field(s.n_b, v=np.outer(np.ones(s.n_b), e))).max() <= 1e-11 * scale
        w = np.zeros(3); w[c] = 1.0
        assert np.abs(Kd @ _field(s.n_b, v=np.cross(w, s.xyz))).max() <= 1e-11 * scale * np.abs(s.xyz).max()
    # nothing on fluid-only rows or on pressures
    Kd = Kd.tocsr()
    solid_rows = cor.solid_rows_of(s).astype(bool)
    rows4 = np.repeat(~solid_rows, 4) | np.tile([False, False, False, True], s.n_b)
    assert abs(Kd[rows4]).max() == 0.0


def test_state_form_is_the_fluid_viscous_energy_for_traceless_fields(fsi_free):
    p, s = fsi_free
    prm = asm.params_of(p)
    Ks = _form(s, prm, "state")
    V = _volumes(s)
    sol = s.tsolid.astype(bool)
    rng = np.random.default_rng(5)
    for _ in range(3):
        A = rng.standard_normal((3, 3))
        A -= np.trace(A) / 3.0 * np.eye(3)          # divergence-free: no grad-div or G/D energy
        u = _field(s.n_b, v=s.xyz @ A.T)
        assert u @ (Ks @ u) == pytest.approx(2.0 * p.mu_f * V[~sol].sum() * _dev_sym_sq(A), rel=1e-11)
    # the solid contributes nothing to the state form's velocity block
    u = _field(s.n_b, v=np.outer(np.ones(s.n_b), [0.3, -0.2, 0.5]))
    assert np.abs(Ks @ u).max() <= 1e-12 * abs(Ks).max()


# ------------------------------------------------------------------------- the time step
def _monolithic(K, solid, state, dt, f, am, af, g):
    """y_dot_{n+1} and u_dot_s,{n+1} from the generalized-alpha equations directly: the balance
    equations at y_dot(alpha_m), y(alpha_f), u_s(alpha_f), the kinematic equation on solid rows,
    and y_{n+1} = y_n + dt y_dot_n + gamma dt (y_dot_{n+1} - y_dot_n) for y and u_s."""
    y, yd, us, usd = (state[k].reshape(-1) for k in ("y", "yd", "us", "usd"))
    n4, n3 = y.size, us.size
    nb = n3 // 3
    E = sp.lil_matrix((n4, n3))                     # (u_s) -> (u_s, 0) per block row
    for r in range(nb):
        for c in range(3):
            E[4 * r + c, 3 * r + c] = 1.0
    E = E.tocsr()
    Pv = E.T                                        # (v, p) -> v
    ay = y + dt * (1.0 - g) * yd                    # y_{n+1} = ay + g dt y_dot_{n+1}
    au = us + dt * (1.0 - g) * usd
    F = np.zeros(n4)
    if f is not None:
        F = E @ f.reshape(-1)
    Kr, Ks, Kd = K["rate"], K["state"], K["disp"]
    A11 = am * Kr + af * g * dt * Ks
    A12 = af * g * dt * (Kd @ E)
    b1 = Kr @ F - Kr @ ((1.0 - am) * yd) - Ks @ ((1.0 - af) * y + af * ay) - Kd @ (E @ ((1.0 - af) * us + af * au))
    srow = np.repeat(solid, 3)
    S = sp.diags(srow.astype(float))
    A21 = -af * g * dt * (S @ Pv)
    A22 = sp.diags(np.where(srow, am, 1.0))
    c = (g - 1.0) / g
    b2 = np.where(srow, -(1.0 - am) * usd + Pv @ ((1.0 - af) * y + af * ay), c * usd)
    # Dirichlet dofs (zero rows of the residual parts): keep the predictor's rate
    dirichlet = np.asarray((abs(Kr) + abs(Ks) + abs(Kd)).sum(axis=1)).ravel() == 0.0
    A11 = A11.tolil()
    A12 = A12.tolil()
    for i in np.nonzero(dirichlet)[0]:
        A11.rows[i], A11.data[i] = [i], [1.0]
        A12.rows[i], A12.data[i] = [], []
    b1 = np.where(dirichlet, c * yd, b1)
    M = sp.bmat([[A11.tocsr(), A12.tocsr()], [A21, A22]]).tocsc()
    x = spla.spsolve(M, np.concatenate([b1, b2]))
    yd1, usd1 = x[:n4], x[n4:]
    return dict(yd=yd1, y=ay + g * dt * yd1, usd=usd1, us=au + g * dt * usd1)


def _stepper(p, s, s_free, dt0, **kw):
    prm = asm.params_of(p)
    return cor.Stepper(cor.assembled_operators(s, prm), cor.solid_rows_of(s),
                       cor.scalar_csr(s.Lrp, s.Lci, s_free.Lval), s.Lmask, s.blk_of_phys, p.rho_inf, dt0, **kw)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _run_against_monolithic(p, s, s_free, steps, corrupt=None):
    st = _stepper(p, s, s_free, 1e-3)
    if corrupt is not None:
        corrupt(st)
    errs = []
    for n, (dt, seed) in enumerate(steps):
        f = synth.rhs(seed, 3 * s.n_b).reshape(-1, 3)
        before = dict(y=st.y.copy(), yd=st.yd.copy(), us=st.us.copy(), usd=st.usd.copy())
        ref = _monolithic(st.operators(dt), st.solid, before, dt, f, st.am, st.af, st.gamma)
        stats = st.step(dt, f)
        assert stats["converged"] and stats["correctors"] == 2, stats
        got = dict(y=st.y, yd=st.yd, us=st.us, usd=st.usd)
        errs.append({k: _rel(got[k].reshape(-1), ref[k]) for k in ref})
        # the kinematic equation holds at the new state
        Rk = st.kinematic_residual(before["usd"] + st.am * (st.usd - before["usd"]),
                                   before["y"] + st.af * (st.y - before["y"]))
        assert np.abs(Rk).max() <= 1e-12 * max(np.abs(st.y[:, :3]).max(), 1e-300)
    return st, errs


def test_multicorrector_reaches_the_generalized_alpha_solution(fsi, fsi_free):
    p, s = fsi
    _, s_free = fsi_free
    steps = [(1e-3, 11), (1e-3, 12), (5e-4, 13), (5e-4, 14)]
    st, errs = _run_against_monolithic(p, s, s_free, steps)
    for e in errs:
        print("[oracle] step errors vs monolithic", {k: f"{v:.1e}" for k, v in e.items()})
        assert max(e.values()) <= 1e-9, e
    assert np.abs(st.us).max() > 0 and np.abs(st.mu).max() > 0
    # mesh: Dirichlet data on solid nodes, the extension elsewhere, and the scheme's
    # u_hat_{n+1} = u_hat_n + dt v_hat_n + gamma dt (v_hat_{n+1} - v_hat_n) over one more step
    mu0, mv0 = st.mu.copy(), st.mv.copy()
    st.step(5e-4, synth.rhs(15, 3 * s.n_b).reshape(-1, 3))
    dt, g = 5e-4, st.gamma
    assert _rel(st.mu, mu0 + dt * mv0 + g * dt * (st.mv - mv0)) <= 1e-12
    d = s.Lmask.astype(bool)
    sol = st.solid[s.blk_of_phys]
    assert np.array_equal(st.mu[d & sol], st.us[s.blk_of_phys[d & sol]])
    assert np.all(st.mu[d & ~sol] == 0.0)
    Lf = cor.scalar_csr(s.Lrp, s.Lci, s_free.Lval)
    r = (Lf @ st.mu)[~d]
    assert np.abs(r).max() <= 1e-10 * np.abs(Lf).max() * np.abs(st.mu).max()


def test_monolithic_check_catches_a_wrong_kinematic_sign(fsi, fsi_free):
    p, s = fsi
    _, s_free = fsi_free

    def corrupt(st):
        good = st.kinematic_residual
        st.kinematic_residual = lambda usd_am, y_af: -good(usd_am, y_af)
    with pytest.raises(AssertionError):
        _run_against_monolithic(p, s, s_free, [(1e-3, 11), (1e-3, 12)], corrupt=corrupt)


def _ode_stepper(rho, k, lam, rho_inf, dt):
    """One block row: an oscillator rho v_dot + k u = 0, u_dot = v per velocity component and a
    decaying mode p_dot + lam p = 0; one Dirichlet mesh node that follows the solid."""
    rate = sp.diags([rho, rho, rho, 1.0]).tocsr()
    state = sp.diags([0.0, 0.0, 0.0, lam]).tocsr()
    disp = sp.diags([k, k, k, 0.0]).tocsr()

    def ops(dt):
        am, af, g = asm.genalpha(rho_inf)
        ct = am / (af * g * dt)
        return {"tangent": (ct * rate + state + disp / ct).tocsr(), "rate": rate, "state": state, "disp": disp}
    return cor.Stepper(ops, np.array([1], np.uint8), sp.csr_matrix(np.ones((1, 1))), np.array([1], np.uint8),
                       np.array([0], np.int32), rho_inf, dt, tol_R=1e-12, tol_A=1e-300)


def _ode_run(rho_inf, nsteps, T=1.0, rho=2.0, k=8.0 * np.pi ** 2, lam=1.5):
    dt = T / nsteps
    st = _ode_stepper(rho, k, lam, rho_inf, dt)
    u0, v0, p0 = np.array([1.0, 0.5, -0.3]), np.array([0.0, 0.2, 0.1]), 1.0
    st.us[0], st.usd[0] = u0, v0
    st.y[0, :3], st.yd[0, :3] = v0, -(k / rho) * u0
    st.y[0, 3], st.yd[0, 3] = p0, -lam * p0
    energy = []
    for _ in range(nsteps):
        stats = st.step(dt)
        assert stats["correctors"] == 2
        energy.append(0.5 * rho * st.y[0, :3] @ st.y[0, :3] + 0.5 * k * st.us[0] @ st.us[0])
    w = np.sqrt(k / rho)
    u_ex = u0 * np.cos(w * T) + v0 / w * np.sin(w * T)
    p_ex = p0 * np.exp(-lam * T)
    return st, np.linalg.norm(st.us[0] - u_ex), abs(st.y[0, 3] - p_ex), np.array(energy)


@pytest.mark.parametrize("rho_inf", [0.0, 0.5, 1.0])
def test_second_order_in_time(rho_inf):
    e_u, e_p = [], []
    for n in (200, 400, 800):
        _, eu, ep, _ = _ode_run(rho_inf, n)
        e_u.append(eu); e_p.append(ep)
    ru = [e_u[i] / e_u[i + 1] for i in range(2)]
    rp = [e_p[i] / e_p[i + 1] for i in range(2)]
    print(f"[oracle] rho_inf={rho_inf} displacement errors {e_u} ratios {ru}; pressure ratios {rp}")
    # halving dt divides the error by about four (the coarsest pair may still be pre-asymptotic)
    assert all(3.6 <= r <= 4.6 for r in ru + rp), (ru, rp)
    assert 3.7 <= ru[-1] <= 4.3 and 3.7 <= rp[-1] <= 4.3, (ru, rp)
    # and the mesh node follows the solid displacement
    st, _, _, _ = _ode_run(rho_inf, 10)
    assert np.array_equal(st.mu[0], st.us[0])


def test_energy_conserved_without_dissipation():
    _, _, _, E = _ode_run(1.0, 300)
    assert np.abs(E / E[0] - 1.0).max() <= 1e-12


def _amplification(rho_inf, wdt, rho=2.0, k=8.0 * np.pi ** 2):
    """The one-step map of (u, v, u_dot, v_dot) of one oscillator component, column by column."""
    dt = wdt / np.sqrt(k / rho)
    A = np.zeros((4, 4))
    for j in range(4):
        st = _ode_stepper(rho, k, 1.0, rho_inf, dt)
        e = np.zeros(4); e[j] = 1.0
        st.us[0, 0], st.y[0, 0], st.usd[0, 0], st.yd[0, 0] = e
        st.step(dt)
        A[:, j] = [st.us[0, 0], st.y[0, 0], st.usd[0, 0], st.yd[0, 0]]
    return np.abs(np.linalg.eigvals(A))


@pytest.mark.parametrize("rho_inf", [0.0, 0.3, 0.5, 0.8, 1.0])
def test_spectral_radius_at_the_highest_mode_is_rho_inf(rho_inf):
    # rho_inf is the spectral radius of the amplification matrix as omega dt -> infinity
    # (Sec. 3.4); the eigenvalues there nearly coincide, so they approach it as (omega dt)^-1/2
    lam = _amplification(rho_inf, 1e6)
    assert np.abs(lam - rho_inf).max() <= 2e-3, lam
    if rho_inf == 1.0:
        assert np.abs(_amplification(1.0, 0.1) - 1.0).max() <= 1e-12
    else:
        # the resolved mode is nearly undamped
        assert 1.0 - 1e-4 <= _amplification(rho_inf, 0.1).max() <= 1.0


def test_harmonic_extension_of_constant_data(fsi, fsi_free):
    _, s = fsi
    _, s_free = fsi_free
    Lf = cor.scalar_csr(s.Lrp, s.Lci, s_free.Lval)
    c = np.array([0.3, -1.2, 2.5])
    uD = np.tile(c, (s.n_phys, 1))
    u = cor.harmonic_extension(Lf, s.Lmask, uD)
    assert np.abs(u - c).max() <= 1e-12
