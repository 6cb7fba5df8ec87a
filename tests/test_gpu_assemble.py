"""GPU parity of the device tangent assembly (scr_assembler_create / scr_assemble_tangent) with
the FP64 oracle (oracle/assembly.py), through the C ABI.

Bar: every block within 1e-12 of the largest entry of its block row of the oracle's matrix (the
two sum the same element contributions in a different arithmetic arrangement; the entries span
several orders of magnitude within a row, so a row-relative bound is the meaningful one).  The
device result is bitwise reproducible.  At the full cfg1 size: every interface row and 10,000
random rows against the oracle (the oracle assembles only the elements touching them), every row
against the generator's matrix to the same bar (a consistency check: the device element arithmetic
follows the generator's), and a solve on the assembled matrix."""
import time

import numpy as np
import pytest

import synth
from oracle import assembly as asm

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


def tparams(scr, p, **over):
    d = asm.params_of(p)
    d.update(over)
    return scr.tangent_params(**d)


def create(scr, ctx, s, p, rp=None, ci=None, tv=None, xyz=None, **over):
    print(f"[gpu] assembler n_b={s.n_b} n_tets={s.n_tets} {over}", flush=True)
    return scr.scr_assembler_create(ctx, dev(s.tv if tv is None else tv), dev(s.tp), dev(s.tsolid),
                                    dev(s.rp if rp is None else rp), dev(s.ci if ci is None else ci),
                                    dev(s.xyz if xyz is None else xyz), dev(s.mask), tparams(scr, p, **over))


def gpu_tangent(scr, a, u=None):
    val = torch.empty(16 * a.nnzb, dtype=torch.float64, device="cuda")
    scr.scr_assemble_tangent(a, None if u is None else dev(u), val)
    return val


def row_rel_err(s, got, ref, rows=None):
    rowof = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    bmax = np.abs(ref).reshape(-1, 16).max(1)
    rmax = np.zeros(s.n_b)
    np.maximum.at(rmax, rowof, bmax)
    d = np.abs(got - ref).reshape(-1, 16).max(1) / np.where(rmax[rowof] > 0, rmax[rowof], 1.0)
    if rows is not None:
        sel = np.zeros(s.n_b, bool); sel[rows] = True
        d = d[sel[rowof]]
    return d.max()


SMALL = dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)


@pytest.mark.parametrize("kw,over", [
    (dict(SMALL), {}),
    (dict(SMALL, u_max=30.0), {}),
    (dict(SMALL, u_max=30.0, apply_bc=0), dict(vms_dt_coupling=1)),
    (dict(SMALL, u_max=30.0), dict(terms=asm.CONV | asm.GD)),
    (dict(mode=1, m_core=5, n_bl=4, nz=4, R=0.5, box_solid=1, apply_bc=0), {}),
    (dict(mode=1, m_core=5, n_bl=4, nz=4, R=0.5, u_max=10.0), {}),
])
def test_small_parity(scr, ctx, kw, over):
    p = synth.default_params(**kw)
    s = synth.generate(p, tets=True)
    u = s.uadv if p.u_max else None
    prm = asm.params_of(p); prm.update(over)
    ref = asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, prm, u=u)
    a = create(scr, ctx, s, p, **over)
    v1 = gpu_tangent(scr, a, u)
    v2 = gpu_tangent(scr, a, u)
    got = host(v1).reshape(-1, 4, 4)
    err = row_rel_err(s, got, ref)
    print(f"[gpu]   row-relative error {err:.2e}", flush=True)
    assert err <= 1e-12
    assert torch.equal(v1, v2)
    a.destroy()


def test_cfg0_advective_assembly_then_setup_update_and_solve(scr, ctx):
    p = synth.cfg0_params()
    p.u_max = 30.0
    s = synth.generate(p, tets=True)
    ref = asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, asm.params_of(p), u=s.uadv)
    a = create(scr, ctx, s, p)
    val = gpu_tangent(scr, a, s.uadv)
    assert row_rel_err(s, host(val).reshape(-1, 4, 4), ref) <= 1e-12
    # the assembled values feed the solver directly
    rp, ci = dev(s.rp), dev(s.ci)
    h = scr.amg_setup(ctx, scr.SCR_SYSTEM, rp, ci, val, dev(s.xyz.reshape(-1)))
    b = synth.rhs(0, 4 * s.n_b, s.mask)
    x = torch.zeros(4 * s.n_b, dtype=torch.float64, device="cuda")
    rc, st = scr.scr_solve(h, dev(b), x)
    xr = host(x)
    Kx = np.zeros((s.n_b, 4))
    rowof = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    np.add.at(Kx, rowof, np.einsum("qij,qj->qi", ref, xr.reshape(-1, 4)[s.ci]))
    assert rc == 0 and np.linalg.norm(b - Kx.reshape(-1)) <= 1e-8 * np.linalg.norm(b)
    # a new advective state: assemble again, numeric re-setup, solve
    val2 = gpu_tangent(scr, a, 0.5 * s.uadv)
    ref2 = asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, asm.params_of(p), u=0.5 * s.uadv)
    assert row_rel_err(s, host(val2).reshape(-1, 4, 4), ref2) <= 1e-12
    scr.amg_update(h, rp, ci, val2)
    x2 = torch.zeros_like(x)
    rc2, _ = scr.scr_solve(h, dev(b), x2)
    Kx[:] = 0.0
    np.add.at(Kx, rowof, np.einsum("qij,qj->qi", ref2, host(x2).reshape(-1, 4)[s.ci]))
    assert rc2 == 0 and np.linalg.norm(b - Kx.reshape(-1)) <= 1e-8 * np.linalg.norm(b)
    h.destroy()
    a.destroy()


def test_invalid_meshes_and_patterns_are_rejected(scr, ctx):
    p = synth.default_params(**SMALL)
    s = synth.generate(p, tets=True)
    tv = s.tv.copy(); tv[3, 2] = s.n_b
    with pytest.raises(scr.ScrError) as e:
        create(scr, ctx, s, p, tv=tv)
    assert e.value.status == scr.SCR_E_INVALID
    xyz = s.xyz.copy(); xyz[s.tv[0, 1]] = xyz[s.tv[0, 0]]
    with pytest.raises(scr.ScrError) as e:
        create(scr, ctx, s, p, xyz=xyz)
    assert e.value.status == scr.SCR_E_INVALID and "degenerate" in str(e.value)
    # drop one coupled off-diagonal block of row tv[0,0]
    r, c = s.tv[0, 0], s.tv[0, 1]
    q = s.rp[r] + int(np.nonzero(s.ci[s.rp[r]:s.rp[r + 1]] == c)[0][0])
    ci = np.delete(s.ci, q)
    rp = s.rp.copy(); rp[r + 1:] -= 1
    with pytest.raises(scr.ScrError) as e:
        create(scr, ctx, s, p, rp=rp, ci=ci)
    assert e.value.status == scr.SCR_E_INVALID and "pattern" in str(e.value)
    ci = s.ci.copy(); ci[s.rp[r]], ci[s.rp[r] + 1] = ci[s.rp[r] + 1], ci[s.rp[r]]
    with pytest.raises(scr.ScrError) as e:
        create(scr, ctx, s, p, ci=ci)
    assert e.value.status == scr.SCR_E_INVALID
    with pytest.raises(scr.ScrError):
        create(scr, ctx, s, p, dt=0.0)
    # the valid inputs still work after the rejections
    a = create(scr, ctx, s, p)
    assert row_rel_err(s, host(gpu_tangent(scr, a)).reshape(-1, 4, 4), s.val) <= 1e-12
    a.destroy()


@pytest.fixture(scope="module")
def cfg1():
    p = synth.cfg1_params()
    p.u_max = 30.0
    return p, synth.generate(p, tets=True)


def test_cfg1_full_size(scr, ctx, cfg1):
    p, s = cfg1
    a = create(scr, ctx, s, p)
    u = dev(s.uadv)
    val = torch.empty(16 * a.nnzb, dtype=torch.float64, device="cuda")
    scr.scr_assemble_tangent(a, u, val)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        scr.scr_assemble_tangent(a, u, val)
    torch.cuda.synchronize()
    print(f"[gpu]   cfg1 assembly {1e3 * (time.perf_counter() - t0) / 5:.2f} ms", flush=True)
    got = host(val).reshape(-1, 4, 4)
    # every row against the generator's matrix: a consistency check with the matrices the solver
    # tests use, not an independent one (the device element arithmetic follows the generator's)
    assert row_rel_err(s, got, s.val) <= 1e-12
    # the independent check, against the oracle: every interface row and its duplicate (where the
    # fluid and solid forms meet), 10,000 random rows, the first and last rows (about 17 % of the
    # rows; the oracle assembles only the elements touching them)
    rng = np.random.default_rng(7)
    iface = np.nonzero(s.kind >= 2)[0]
    rows = np.unique(np.concatenate([rng.choice(s.n_b, 10000, replace=False), iface, [0, s.n_b - 1]]))
    print(f"[gpu]   oracle rows {rows.size} of {s.n_b}", flush=True)
    ref = asm.tangent(s.tv, s.tp, s.tsolid, s.xyz, s.rp, s.ci, s.mask, asm.params_of(p), u=s.uadv, rows=rows)
    assert row_rel_err(s, got, ref, rows=rows) <= 1e-12
    a.destroy()
