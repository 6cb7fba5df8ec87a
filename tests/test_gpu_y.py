"""GPU parity on the Y-bifurcation voxel workload (parent radius 1, daughters 0.7 at seeded angles,
wall to 1.2x the local radius, staircase fluid/solid interface).

* A small Y (about 4k nodes): every level of AMG(A), AMG(S^) and AMG(L) against the oracle's
  hierarchies (patterns and aggregates bit-exact, values to 1e-11); FP64 and mixed solves to a
  1e-8 true residual (recomputed by the oracle's SpMV) within 1e-6 of the oracle's solution at
  1e-11; the mesh-motion solve within 1e-7 of the oracle's.
* The full-size Y (about 4.0M nodes, 3.9M+ block rows): level-0 strength flags and aggregates of
  A bit-exact against the oracle's own functions; mixed and FP64 solves to 1e-8 (oracle SpMV)
  agreeing to 1e-6; the mesh-motion solve to 1e-8 on all three right-hand sides.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import assert_fields
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


def _setup(scr, ctx, s, **kw):
    print(f"[gpu] Y amg_setup n_b={s.n_b} nnzb={s.nnzb} {kw}", flush=True)
    return scr.amg_setup(ctx, scr.SCR_SYSTEM, dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)), dev(s.xyz.reshape(-1)),
                         scr.amg_opts(**kw))


def _rel(s, b, x):
    return np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, x)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def ysmall():
    return synth.generate(synth.y_params(h=0.25, seed=0))


def test_y_small_hierarchies_and_solves(scr, ctx, ysmall):
    s = ysmall
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    h = _setup(scr, ctx, s)
    _compare_hierarchy(h, 0, o.amgA)
    _compare_hierarchy(h, 1, o.amgS)
    h.destroy()
    b = synth.rhs(21, 4 * s.n_b, s.mask)
    # the reference as tight as rounding allows here (the floor is near 1e-12)
    xo, rco, sto = o.solve(b, oracle.solve_opts(tol=1e-11, max_it=12))
    assert sto["rel_res_true"] <= 1e-11
    for precision in (0, 1, 2):
        h = _setup(scr, ctx, s, precision=precision)
        x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
        rc, st = scr.scr_solve(h, dev(b), x)
        xg = x.cpu().numpy()
        rel = _rel(s, b, xg)
        print(f"[gpu] Y small precision={precision} rc={rc} outer={st['outer_it']} its_A={st['its_A']} "
              f"its_S={st['its_S']} rel={rel:.2e}", flush=True)
        assert rc == 0 and rel <= 1e-8
        assert_fields(xg, xo, 1e-6, f"Y small precision={precision}")
        h.destroy()


def test_y_small_mesh_motion(scr, ctx, ysmall):
    s = ysmall
    h = scr.amg_setup(ctx, scr.MESH_SYSTEM, dev(s.Lrp), dev(s.Lci), dev(s.Lval))
    m = oracle.Mesh(s.Lrp, s.Lci, s.Lval)
    _compare_hierarchy(h, 2, m.amg)
    b = synth.rhs(22, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    xo, rc, its, rel = m.solve(b, tol=1e-12)
    x = torch.zeros(3 * s.n_phys, dtype=torch.float64, device="cuda")
    rc, st = scr.mesh_motion_solve(h, dev(b), x, scr.solve_opts(tol=1e-10, max_it=500))
    xg = x.cpu().numpy()
    assert rc == 0 and np.linalg.norm(xg - xo) <= 1e-7 * np.linalg.norm(xo)
    h.destroy()


@pytest.mark.timeout(900)
def test_y_full_size(scr, ctx):
    p = synth.cfg4_params()
    print(f"[gpu] Y full: generating (h={p.y_h:.5f})", flush=True)
    s = synth.generate(p)
    print(f"[gpu] Y full: nodes={s.n_phys} n_b={s.n_b} nnzb={s.nnzb} iface={s.n_iface}", flush=True)
    A = np.ascontiguousarray(s.val[:, :3, :3])
    flags, iso = oracle.strength(s.rp, s.ci, A, 0.08)
    root = oracle.mis2(s.rp, s.ci, flags, iso, 0, 0)
    na, agg = oracle.aggregate(s.rp, s.ci, flags, iso, root, 0, 0)
    del A
    b = synth.rhs(40, 4 * s.n_b, s.mask)
    xs = {}
    for precision in (1, 0):
        h = _setup(scr, ctx, s, precision=precision)
        if precision == 1:
            assert np.array_equal(h.hier_level_copy(0, 0, "strong"), flags)
            assert np.array_equal(h.hier_level_copy(0, 0, "agg"), agg)
            assert h.hier_level_info(0, 0)["nagg"] == na
        x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
        rc, st = scr.scr_solve(h, dev(b), x)
        xs[precision] = x.cpu().numpy()
        rel = _rel(s, b, xs[precision])
        print(f"[gpu] Y full precision={precision} rc={rc} outer={st['outer_it']} its_A={st['its_A']} "
              f"its_S={st['its_S']} vA={st['vcycles_A']} rel={rel:.2e} setup={st['t_setup_ms']:.0f}ms "
              f"solve={st['t_solve_ms']:.0f}ms", flush=True)
        assert rc == 0 and rel <= 1e-8
        h.destroy()
    assert_fields(xs[1], xs[0], 1e-6, "Y full, mixed against FP64")
    hm = scr.amg_setup(ctx, scr.MESH_SYSTEM, dev(s.Lrp), dev(s.Lci), dev(s.Lval), None, scr.amg_opts(precision=1))
    bm = synth.rhs(41, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    xm = torch.zeros(3 * s.n_phys, dtype=torch.float64, device="cuda")
    rcm, stm = scr.mesh_motion_solve(hm, dev(bm), xm)
    xmg = xm.cpu().numpy()
    print(f"[gpu] Y full mesh rc={rcm} its={stm['mesh_its']}", flush=True)
    assert rcm == 0
    for c in range(3):
        bc = bm[c::3]
        assert np.linalg.norm(bc - oracle.bsr_spmv(s.Lrp, s.Lci, s.Lval, xmg[c::3])) <= 1e-8 * np.linalg.norm(bc)
    hm.destroy()
