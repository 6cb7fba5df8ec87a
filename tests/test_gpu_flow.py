"""GPU parity on the advective (nonsymmetric) systems and with the outlet resistance coupling,
through the C ABI, against the FP64 oracle.

Bars as in the setup/solve parity tests: patterns, strength flags and aggregates bit-exact;
hierarchy values within 1e-11; operators within 1e-13 of the largest entry (1e-12 where the
outlet dot products are reduced in a different order); solves to a 1e-8 true residual with FP64
iteration counts equal to the oracle's and ||x - x_oracle|| <= 1e-6 ||x_oracle|| against the
oracle solved to 1e-12; with the coupling, solves to 1e-11 against the Woodbury update of the
plain system's dense LU."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import assert_fields, bsr_to_dense
from tests.test_gpu_parity import _compare_hierarchy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def flow_small():
    kw = dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)
    return synth.generate(synth.default_params(u_max=30.0, **kw))


@pytest.fixture(scope="module")
def flow_cfg0():
    p = synth.cfg0_params()
    p.u_max = 30.0
    return synth.generate(p)


def setup(scr, ctx, s, **kw):
    print(f"[gpu] amg_setup n_b={s.n_b} {kw}", flush=True)
    return scr.amg_setup(ctx, scr.SCR_SYSTEM, dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)), dev(s.xyz.reshape(-1)),
                         scr.amg_opts(**kw))


def two_outlets(s):
    blk, a = s.outlets[0]
    h = len(blk) // 2
    return [(blk[:h], a[:h]), (blk[h:], a[h:])], np.array([1.0e3, 4.0e3])


def test_advective_hierarchy_parity(scr, ctx, flow_small):
    s = flow_small
    h = setup(scr, ctx, s, coarse_max=60)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(coarse_max=60))
    _compare_hierarchy(h, 0, o.amgA)
    _compare_hierarchy(h, 1, o.amgS)
    h.destroy()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_advective_cfg0_solve_parity(scr, ctx, flow_cfg0, precision):
    s = flow_cfg0
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    b = synth.rhs(0, 4 * s.n_b, s.mask)
    xo, rco, sto = o.solve(b, oracle.solve_opts(tol=1e-8))
    xt, rct, _ = o.solve(b, oracle.solve_opts(tol=1e-12))
    assert rco == 0 and rct == 0
    h = setup(scr, ctx, s, precision=precision)
    x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    rc, st = scr.scr_solve(h, dev(b), x)
    xg = host(x)
    rel = np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, xg)) / np.linalg.norm(b)
    print(f"[gpu]   outer gpu={st['outer_it']} oracle={sto['outer_it']} rel={rel:.2e}", flush=True)
    assert rc == 0 and rel <= 1e-8
    if precision == 0:
        assert st["outer_it"] == sto["outer_it"]
    assert_fields(xg, xt, 1e-6, f"advective cfg0 precision={precision}")
    h.destroy()


def test_outlet_operators_match_the_oracle(scr, ctx, flow_small):
    s = flow_small
    outlets, m = two_outlets(s)
    h = setup(scr, ctx, s, coarse_max=60)
    scr.set_outlets(h, outlets, m)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(coarse_max=60))
    o.set_outlets(outlets, m)
    rng = np.random.default_rng(0)
    for op, n in (("K", 4 * s.n_b), ("A", 3 * s.n_b)):
        x = rng.uniform(-1, 1, n)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        scr.scr_apply(h, op, dev(x), y)
        yo = o.apply(op, x)
        assert np.abs(host(y) - yo).max() <= 1e-12 * np.abs(yo).max(), op
    tight = dict(tol_I=1e-13, max_it_I=400)
    xp = rng.normal(size=s.n_b)
    y = torch.empty(s.n_b, dtype=torch.float64, device="cuda")
    scr.scr_apply(h, "S", dev(xp), y, scr.solve_opts(**tight))
    yo = o.apply("S", xp, oracle.solve_opts(**tight))
    assert np.linalg.norm(host(y) - yo) <= 1e-9 * np.linalg.norm(yo)
    h.destroy()


def test_outlet_coupled_solve_is_the_woodbury_update(scr, ctx, flow_small):
    s = flow_small
    outlets, m = two_outlets(s)
    Kd = bsr_to_dense(s.rp, s.ci, s.val)
    U = np.zeros((2, s.n_b, 4))
    for k, (blk, a) in enumerate(outlets):
        U[k][blk, :3] = a
    U = U.reshape(2, -1).T
    b = synth.rhs(3, 4 * s.n_b, s.mask)
    y = np.linalg.solve(Kd, b)
    Z = np.linalg.solve(Kd, U)
    xw = y - Z @ np.linalg.solve(np.diag(1.0 / m) + U.T @ Z, U.T @ y)
    for precision in (0, 1, 2):
        h = setup(scr, ctx, s, precision=precision)
        scr.set_outlets(h, outlets, m)
        x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
        rc, st = scr.scr_solve(h, dev(b), x, scr.solve_opts(tol=1e-11))
        assert rc == 0
        assert_fields(host(x), xw, 1e-9, f"Woodbury precision={precision}")
        h.destroy()
    assert np.linalg.norm(y - xw) > 1e-5 * np.linalg.norm(xw)


def test_outlet_coupled_cfg0_solve_parity(scr, ctx, flow_cfg0):
    s = flow_cfg0
    blk, a = s.outlets[0]
    outlets, m = [(blk, a)], np.array([2.0e3])
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    o.set_outlets(outlets, m)
    b = synth.rhs(1, 4 * s.n_b, s.mask)
    xo, rco, sto = o.solve(b, oracle.solve_opts(tol=1e-8))
    xt, _, _ = o.solve(b, oracle.solve_opts(tol=1e-12))
    h = setup(scr, ctx, s)
    scr.set_outlets(h, outlets, m)
    x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    rc, st = scr.scr_solve(h, dev(b), x)
    print(f"[gpu]   outer gpu={st['outer_it']} oracle={sto['outer_it']}", flush=True)
    assert rc == 0 and rco == 0 and st["outer_it"] == sto["outer_it"]
    assert st["rel_res_true"] <= 1e-8
    assert_fields(host(x), xt, 1e-6, "outlet-coupled cfg0")
    # the coupling survives a numeric re-setup with the same values
    scr.amg_update(h, dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)))
    x2 = torch.zeros_like(x)
    rc2, st2 = scr.scr_solve(h, dev(b), x2)
    assert rc2 == 0 and np.array_equal(host(x2), host(x))
    h.destroy()


def test_invalid_outlets_keep_the_previous_coupling(scr, ctx, flow_small):
    s = flow_small
    outlets, m = two_outlets(s)
    h = setup(scr, ctx, s, coarse_max=60)
    scr.set_outlets(h, outlets, m)
    b = synth.rhs(4, 4 * s.n_b, s.mask)
    x0 = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    scr.scr_solve(h, dev(b), x0)
    blk0, a0 = outlets[0]
    bad = [
        ([(blk0, a0), (blk0[:1], a0[:1])], [1.0, 1.0]),              # a row in two outlets
        ([(np.array([s.n_b], np.int32), a0[:1])], [1.0]),           # row out of range
        ([(blk0, np.where(np.arange(a0.size).reshape(a0.shape) == 0, np.nan, a0))], [1.0]),
        ([(blk0, a0)], [np.inf]),
    ]
    for outs, mm in bad:
        with pytest.raises(scr.ScrError) as e:
            scr.set_outlets(h, outs, mm)
        assert e.value.status == scr.SCR_E_INVALID
    x1 = torch.zeros_like(x0)
    scr.scr_solve(h, dev(b), x1)
    assert np.array_equal(host(x0), host(x1))
    # removing the coupling gives the plain solve
    scr.set_outlets(h, [], [])
    hp = setup(scr, ctx, s, coarse_max=60)
    x2 = torch.zeros_like(x0); x3 = torch.zeros_like(x0)
    scr.scr_solve(h, dev(b), x2)
    scr.scr_solve(hp, dev(b), x3)
    assert np.array_equal(host(x2), host(x3))
    hm = scr.amg_setup(ctx, scr.MESH_SYSTEM, dev(s.Lrp), dev(s.Lci), dev(s.Lval))
    with pytest.raises(scr.ScrError):
        scr.set_outlets(hm, outlets, m)
    h.destroy(); hp.destroy(); hm.destroy()
