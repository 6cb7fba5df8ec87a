"""SIMPLE and SIMPLEC block preconditioners (Sec. 5.2.1) on the GPU against the oracle: the lumped
diagonal and S^ (patterns bit-exact), AMG(S^) built on the SIMPLEC S^, the preconditioner's
action with tight block solves, and full FGMRES solves (FP64 and mixed) with the oracle's
iteration counts in FP64."""
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
    print(f"[gpu] amg_setup n_b={s.n_b} {kw}", flush=True)
    return scr.amg_setup(ctx, scr.SCR_SYSTEM, dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)), dev(s.xyz.reshape(-1)),
                         scr.amg_opts(**kw))


@pytest.mark.parametrize("schur_diag", [0, 1])
def test_lumped_diagonal_schur_and_hierarchy(scr, ctx, small_fsi, cfg0, schur_diag):
    for s in (small_fsi, cfg0):
        h = _setup(scr, ctx, s, schur_diag=schur_diag)
        o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(schur_diag=schur_diag))
        d = torch.zeros(3 * s.n_b, dtype=torch.float64, device="cuda")
        scr.scr_apply(h, "d", torch.zeros_like(d), d)
        assert np.array_equal(d.cpu().numpy(), o.apply("d", np.zeros(3 * s.n_b)))
        rp, ci, v = h.matrix_copy("Shat")
        orp, oci, ov = o.matrix("Shat")
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert np.abs(v - ov).max() <= 1e-13 * np.abs(ov).max()
        _compare_hierarchy(h, 1, o.amgS)
        h.destroy()


@pytest.mark.parametrize("schur_diag", [0, 1])
def test_simple_action_with_tight_block_solves(scr, ctx, small_fsi, schur_diag):
    s = small_fsi
    h = _setup(scr, ctx, s, schur_diag=schur_diag)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(schur_diag=schur_diag))
    r = np.random.default_rng(12).normal(size=4 * s.n_b)
    tight_g = scr.solve_opts(tol_A=1e-13, tol_S=1e-13, max_it_A=400, max_it_S=400)
    tight_o = oracle.solve_opts(tol_A=1e-13, tol_S=1e-13, max_it_A=400, max_it_S=400)
    y = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    scr.scr_apply(h, "SIMPLE", dev(r), y, tight_g)
    yo = o.apply("SIMPLE", r, tight_o)
    assert np.linalg.norm(y.cpu().numpy() - yo) <= 1e-9 * np.linalg.norm(yo)
    h.destroy()


@pytest.mark.parametrize("schur_diag", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_simple_solves_match_oracle(scr, ctx, cfg0, schur_diag, precision):
    s = cfg0
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(schur_diag=schur_diag))
    b = synth.rhs(13, 4 * s.n_b, s.mask)
    xo, rco, sto = o.solve(b, oracle.solve_opts(tol=1e-8, precond=1))
    xt, rct, stt = o.solve(b, oracle.solve_opts(tol=1e-12, precond=1))
    assert rco == 0 and rct == 0
    h = _setup(scr, ctx, s, schur_diag=schur_diag, precision=precision)
    x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    rc, st = scr.scr_solve(h, dev(b), x, scr.solve_opts(precond=scr.SCR_PRECOND_SIMPLE))
    xg = x.cpu().numpy()
    rel = np.linalg.norm(b - oracle.bsr_spmv(s.rp, s.ci, s.val, xg)) / np.linalg.norm(b)
    print(f"[gpu] SIMPLE schur_diag={schur_diag} precision={precision}: rc={rc} outer={st['outer_it']} "
          f"its_A={st['its_A']} its_S={st['its_S']} calls_I={st['calls_I']} rel={rel:.2e}; "
          f"oracle outer={sto['outer_it']} its_A={sto['its_A']} its_S={sto['its_S']}", flush=True)
    assert rc == 0 and rel <= 1e-8 and st["calls_I"] == 0
    assert_fields(xg, xt, 1e-6, f"SIMPLE schur_diag={schur_diag} precision={precision}")
    if precision == 0:
        for k in ("outer_it", "its_A", "its_S", "calls_A", "calls_S"):
            assert st[k] == sto[k], k
    h.destroy()
