"""GPU parity of the device time stepper (scr_stepper_create / scr_step / scr_stepper_state) with
the FP64 oracle of the predictor multi-corrector (oracle/corrector.py), through the C ABI.

The oracle solves each corrector system and the mesh motion exactly (sparse LU); the device solves
them iteratively (with smoothed-aggregation AMG in FP64 and mixed precision, and with the classical
AMG option) (scr_solve to 1e-10, the mesh CG to 1e-12), so every field of the state is
compared per field at 1e-7 relative to its own norm after every step.  The step count of
correctors (2 for this linear model: one Newton step, then the test that passes), the re-setup on
a change of dt and the state copies are checked as well.
"""
import numpy as np
import pytest

import synth
from oracle import assembly as asm
from oracle import corrector as cor

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SMALL = dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)
FIELDS = {"y": ("y", 4), "ydot": ("yd", 4), "u_solid": ("us", 3), "udot_solid": ("usd", 3),
          "u_mesh": ("mu", 3), "v_mesh": ("mv", 3)}


@pytest.fixture(scope="module")
def scr():
    import paper_2206_06996_amd.scr as m
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return m


@pytest.fixture(scope="module")
def ctx(scr):
    c = scr.Context(0)
    yield c
    c.destroy()


@pytest.fixture(scope="module")
def tube():
    p = synth.default_params(**SMALL)
    s = synth.generate(p, tets=True)
    s_free = synth.generate(synth.default_params(apply_bc=0, **SMALL))
    return p, s, s_free


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _pair(scr, ctx, tube, dt0, precision=0, max_correctors=10, amg_type=0):
    p, s, s_free = tube
    print(f"[gpu] stepper n_b={s.n_b} n_L={s.n_phys} dt0={dt0} precision={precision} amg_type={amg_type}", flush=True)
    a = scr.scr_assembler_create(ctx, dev(s.tv), dev(s.tp), dev(s.tsolid), dev(s.rp), dev(s.ci), dev(s.xyz),
                                 dev(s.mask), scr.tangent_params(**asm.params_of(p)))
    solid = cor.solid_rows_of(s)
    st = scr.scr_stepper_create(ctx, a, dev(s.Lrp), dev(s.Lci), dev(s.Lval), dev(s_free.Lval), dev(s.Lmask),
                                dev(s.blk_of_phys), dev(solid), dev(s.xyz.reshape(-1)), dt0,
                                amg=scr.amg_opts(precision=precision, amg_type=amg_type), solve=scr.solve_opts(tol=1e-10),
                                copts=scr.corrector_opts(mesh_tol=1e-12, max_correctors=max_correctors))
    orc = cor.Stepper(cor.assembled_operators(s, asm.params_of(p)), solid, cor.scalar_csr(s.Lrp, s.Lci, s_free.Lval),
                      s.Lmask, s.blk_of_phys, p.rho_inf, dt0, max_correctors=max_correctors)
    return a, st, orc


def _compare(st, orc, tol, what):
    worst = 0.0
    for name, (attr, w) in FIELDS.items():
        g = st.state(name).cpu().numpy().reshape(-1, w)
        r = getattr(orc, attr)
        if name in ("y", "ydot"):
            errs = [np.linalg.norm(g[:, :3] - r[:, :3]) / max(np.linalg.norm(r[:, :3]), 1e-300),
                    np.linalg.norm(g[:, 3] - r[:, 3]) / max(np.linalg.norm(r[:, 3]), 1e-300)]
        else:
            errs = [np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)]
        print(f"[gpu]   {what} {name}: rel err {', '.join(f'{e:.1e}' for e in errs)} "
              f"(|ref| {np.linalg.norm(r):.2e})", flush=True)
        assert max(errs) <= tol, (what, name, errs)
        worst = max(worst, max(errs))
    return worst


@pytest.mark.parametrize("precision,amg_type", [(0, 0), (1, 0), (0, 1)])
def test_steps_match_oracle(scr, ctx, tube, precision, amg_type):
    p, s, _ = tube
    a, st, orc = _pair(scr, ctx, tube, 1e-3, precision, amg_type=amg_type)
    for n, dt in enumerate([1e-3, 1e-3, 5e-4, 5e-4]):
        f = synth.rhs(100 + n, 3 * s.n_b)
        rc, gs = st.step(dt, dev(f))
        os_ = orc.step(dt, f.reshape(-1, 3))
        print(f"[gpu] step {n} dt={dt}: rc={rc} {gs}; oracle {os_}", flush=True)
        assert rc == scr.SCR_OK and gs["converged"] == 1
        assert gs["correctors"] == os_["correctors"] == 2
        assert gs["resetups"] == os_["resetups"] == (1 if n == 2 else 0)
        assert gs["linear_its"] > 0 and gs["mesh_its"] > 0
        assert gs["res0"] == pytest.approx(os_["res0"], rel=1e-9)
        _compare(st, orc, 1e-7, f"step {n}")
    st.destroy()
    a.destroy()


def _random_state(st, orc, s, seed):
    rng = np.random.default_rng(seed)
    m = s.mask.reshape(-1, 4).astype(bool)
    for name, (attr, w) in FIELDS.items():
        n = (s.n_phys if name.endswith("mesh") else s.n_b) * w
        v = rng.standard_normal(n).reshape(-1, w)
        if name in ("y", "ydot"):
            v[m] = 0.0                   # the Dirichlet dofs carry their (homogeneous) data
        st.set_state(name, dev(v.reshape(-1)))
        assert np.array_equal(st.state(name).cpu().numpy(), v.reshape(-1))
        setattr(orc, attr, v.copy())


def test_state_roundtrip_and_a_step_from_a_given_state(scr, ctx, tube):
    p, s, _ = tube
    a, st, orc = _pair(scr, ctx, tube, 1e-3)
    _random_state(st, orc, s, 7)
    f = synth.rhs(5, 3 * s.n_b)
    rc, gs = st.step(1e-3, dev(f))
    os_ = orc.step(1e-3, f.reshape(-1, 3))
    print(f"[gpu] step from a random state: rc={rc} {gs}; oracle {os_}", flush=True)
    assert rc == scr.SCR_OK and gs["correctors"] == os_["correctors"] == 2
    _compare(st, orc, 1e-7, "random start")
    st.destroy()
    a.destroy()


def test_single_corrector_reports_not_converged(scr, ctx, tube):
    p, s, _ = tube
    a, st, orc = _pair(scr, ctx, tube, 1e-3, max_correctors=1)
    _random_state(st, orc, s, 8)
    f = synth.rhs(9, 3 * s.n_b)
    rc, gs = st.step(1e-3, dev(f))
    os_ = orc.step(1e-3, f.reshape(-1, 3))
    print(f"[gpu] one corrector: rc={rc} {gs}; oracle {os_}", flush=True)
    assert rc == scr.SCR_NOT_CONVERGED and gs["converged"] == 0 and not os_["converged"]
    assert gs["correctors"] == 1 and gs["linear_its"] == 0
    # no corrector solve: the predictor, the solid update and the mesh motion only
    _compare(st, orc, 1e-9, "one corrector")
    assert gs["res"] == pytest.approx(os_["res"], rel=1e-10)
    with pytest.raises(scr.ScrError):
        st.step(-1.0)
    buf = dev(np.zeros(4 * s.n_b))
    assert scr.lib().scr_stepper_state(st.ptr, 17, buf.data_ptr(), 0, None) == scr.SCR_E_INVALID
    st.destroy()
    a.destroy()
