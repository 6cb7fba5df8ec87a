"""GPU parity at the full workload sizes (the launch configuration bench.py times).

* cfg1 (300,899 nodes): every level of AMG(A) and AMG(S^) against the oracle's hierarchy
  (aggregates, strength flags, dead dofs and all patterns bit-exact; values to 1e-11); FP64 and both
  mixed forms solved to delta = 1e-8 and compared, velocity and pressure apart, with 2,000 sampled
  entries of each field of the oracle's solution refined towards 1e-11 (oracle/cfg1_reference.json,
  written by oracle/reference_run.py), then refined themselves and compared again; true residuals
  recomputed by the oracle's SpMV; FP64 iteration counts equal to the oracle's; the handle's
  measured peak of device memory within its footprint estimate.
* cfg2 (1.46M nodes): level-0 strength flags and aggregates of A bit-exact against the oracle's own
  functions; FP64 and both mixed forms solved to 1e-8 (oracle SpMV) and compared per field with the
  oracle's refined solution (oracle/cfg2_reference.json); footprint as for cfg1.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests.conftest import ROOT

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REF = os.path.join(ROOT, "oracle", "cfg1_reference.json")


def _complete(path):
    """the reference file exists and holds its last phase (it is rewritten after each phase)"""
    if not os.path.exists(path):
        return False
    try:
        return "xtv_sample" in json.load(open(path))
    except ValueError:
        return False


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


@pytest.fixture(scope="module")
def cfg1():
    return synth.generate(synth.cfg1_params())


def _setup(scr, ctx, s, **kw):
    print(f"[gpu] amg_setup n_b={s.n_b} {kw}", flush=True)
    return scr.amg_setup(ctx, scr.SCR_SYSTEM, dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)), dev(s.xyz.reshape(-1)),
                         scr.amg_opts(**kw))


def test_cfg1_hierarchies_match_oracle(scr, ctx, cfg1):
    from tests.test_gpu_parity import _compare_hierarchy
    h = _setup(scr, ctx, cfg1)
    o = oracle.Scr(cfg1.rp, cfg1.ci, cfg1.val, cfg1.xyz)
    _compare_hierarchy(h, 0, o.amgA)
    _compare_hierarchy(h, 1, o.amgS)
    h.destroy()


def _sampled_field_errors(xg, ref, key):
    """Relative errors of the sampled velocity and pressure entries against the reference's."""
    out = []
    for f in ("v", "p"):
        idx = np.array(ref[f"x{f}_sample_idx"])
        r = np.array(ref[f"{key}{f}_sample"])
        out.append(float(np.linalg.norm(xg[idx] - r) / np.linalg.norm(r)))
    return out


def _solution_against_reference(scr, ctx, s, ref, precision, label):
    """One corrector solve at delta = 1e-8 on the reference's right-hand side, compared per field
    with the oracle's refined solution; then refined as far as the oracle went and compared again."""
    b = synth.rhs(ref["rhs_seed"], 4 * s.n_b, s.mask)
    h = _setup(scr, ctx, s, precision=precision)
    x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    bd = dev(b)
    rc, st = scr.scr_solve(h, bd, x)
    xg = x.cpu().numpy()
    rel8 = np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, xg)) / np.linalg.norm(b)
    ev, ep = _sampled_field_errors(xg, ref, "xt")
    fp = scr.footprint_estimate(scr.SCR_SYSTEM, s.n_b, s.nnzb, scr.amg_opts(precision=precision))
    print(f"[gpu] {label} precision={precision} rc={rc} outer={st['outer_it']} its_A={st['its_A']} its_S={st['its_S']} "
          f"its_I={st['its_I']} rel(oracle SpMV)={rel8:.2e} sampled err vs oracle (refined): velocity {ev:.2e} "
          f"pressure {ep:.2e}; oracle's own 1e-8 solution: {ref['x8_vs_xt_rel']}; oracle counts {ref['stats_1e-8']}; "
          f"peak bytes {h.peak_bytes()} footprint {fp}", flush=True)
    assert rc == 0 and rel8 <= 1e-8
    assert ev <= 1e-6 and ep <= 1e-6
    assert 0 < h.peak_bytes() <= fp
    if precision == 0:
        # same algorithm in the same precision: the same counts as the oracle's own solve
        for k in ("outer_it", "its_A", "its_S", "its_I", "vcycles_A", "vcycles_S"):
            assert st[k] == ref["stats_1e-8"][k], k
    rc, st = scr.scr_solve(h, bd, x, scr.solve_opts(tol=1e-11, max_it=8, use_x0=1))
    xg = x.cpu().numpy()
    rel = np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, xg)) / np.linalg.norm(b)
    ev, ep = _sampled_field_errors(xg, ref, "xt")
    print(f"[gpu] {label} precision={precision} refined: rc={rc} outer={st['outer_it']} rel={rel:.2e} "
          f"(oracle {ref['tight_rel_res']:.2e}) sampled err: velocity {ev:.2e} pressure {ep:.2e}", flush=True)
    assert rel <= max(1e-10, 10 * ref["tight_rel_res"])
    assert ev <= 1e-8 and ep <= 1e-8
    h.destroy()


@pytest.mark.skipif(not _complete(REF), reason="oracle/cfg1_reference.json not generated")
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_cfg1_solution_matches_oracle_samples(scr, ctx, cfg1, precision):
    ref = json.load(open(REF))
    s = cfg1
    _solution_against_reference(scr, ctx, s, ref, precision, "cfg1")
    # mesh motion, same right-hand side seed and tolerance as the reference
    bm = synth.rhs(ref["mesh_rhs_seed"], 3 * s.n_phys, np.repeat(s.Lmask, 3))
    hm = scr.amg_setup(ctx, scr.MESH_SYSTEM, dev(s.Lrp), dev(s.Lci), dev(s.Lval), None,
                       scr.amg_opts(precision=precision))
    xm = torch.zeros(3 * s.n_phys, dtype=torch.float64, device="cuda")
    rcm, stm = scr.mesh_motion_solve(hm, dev(bm), xm, scr.solve_opts(tol=1e-12, max_it=500))
    xmg = xm.cpu().numpy()
    idm = np.array(ref["xm_sample_idx"])
    xms = np.array(ref["xm_sample"])
    errm = np.linalg.norm(xmg[idm] - xms) / np.linalg.norm(xms)
    fpm = scr.footprint_estimate(scr.MESH_SYSTEM, s.n_phys, s.Lci.size, scr.amg_opts(precision=precision))
    print(f"[gpu] cfg1 mesh precision={precision} rc={rcm} its={stm['mesh_its']} err={errm:.2e} "
          f"peak bytes {hm.peak_bytes()} footprint {fpm}", flush=True)
    assert rcm == 0 and errm <= 1e-9
    assert 0 < hm.peak_bytes() <= fpm
    hm.destroy()


REF2 = os.path.join(ROOT, "oracle", "cfg2_reference.json")


@pytest.fixture(scope="module")
def cfg2():
    return synth.generate(synth.cfg2_params())


def test_cfg2_level0_aggregates_match_oracle(scr, ctx, cfg2):
    s = cfg2
    print(f"[gpu] cfg2 n_b={s.n_b} nnzb={s.nnzb}", flush=True)
    A = np.ascontiguousarray(s.val[:, :3, :3])
    flags, iso = oracle.strength(s.rp, s.ci, A, 0.08)
    root = oracle.mis2(s.rp, s.ci, flags, iso, 0, 0)
    na, agg = oracle.aggregate(s.rp, s.ci, flags, iso, root, 0, 0)
    h = _setup(scr, ctx, s)
    assert np.array_equal(h.hier_level_copy(0, 0, "strong"), flags)
    assert np.array_equal(h.hier_level_copy(0, 0, "agg"), agg)
    assert h.hier_level_info(0, 0)["nagg"] == na
    h.destroy()


@pytest.mark.skipif(not _complete(REF2), reason="oracle/cfg2_reference.json not generated")
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_cfg2_solution_matches_oracle_samples(scr, ctx, cfg2, precision):
    ref = json.load(open(REF2))
    assert ref["n_b"] == cfg2.n_b and ref["nnzb"] == cfg2.nnzb
    _solution_against_reference(scr, ctx, cfg2, ref, precision, "cfg2")
