"""Serving (continuous batching) on the GPU: every request's results are the same alone and in the
mix (bitwise: the kernels are deterministic and requests share no state) and solve their systems
(true residuals recomputed by the oracle's SpMV), every request's measured device-memory peak stays
within its admission footprint, admission respects the device-memory budget, oversize requests are
rejected, and a failing request does not disturb the others."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def scr():
    import paper_2206_06996_amd.scr as m
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _systems():
    ps = [synth.tiny_annulus_params(),
          synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0),
          synth.cfg0_params(),
          synth.tube_params(12000, 0.7, 3.0),
          synth.tube_params(25000, 1.3, 6.0)]
    out = []
    for k, p in enumerate(ps):
        s = synth.generate(p)
        nrhs = 1 + k % 3
        out.append(dict(
            K=(dev(s.rp), dev(s.ci), dev(s.val.reshape(-1))), coords=dev(s.xyz.reshape(-1)),
            L=(dev(s.Lrp), dev(s.Lci), dev(s.Lval)),
            b=[dev(synth.rhs(100 * k + c, 4 * s.n_b, s.mask)) for c in range(nrhs)],
            bm=[dev(synth.rhs(100 * k + 50 + c, 3 * s.n_phys, np.repeat(s.Lmask, 3))) for c in range(nrhs)],
            nb=s.n_b, nphys=s.n_phys, sys=s))
    return out


@pytest.fixture(scope="module")
def systems():
    return _systems()


def _alone(scr, ctx, sysd):
    xs, xms = [], []
    h = scr.amg_setup(ctx, scr.SCR_SYSTEM, *sysd["K"], sysd["coords"])
    hm = scr.amg_setup(ctx, scr.MESH_SYSTEM, *sysd["L"])
    for b, bm in zip(sysd["b"], sysd["bm"]):
        x = torch.zeros_like(b); xm = torch.zeros_like(bm)
        rc, _ = scr.scr_solve(h, b, x)
        rcm, _ = scr.mesh_motion_solve(hm, bm, xm)
        assert rc == 0 and rcm == 0
        xs.append(x.cpu().numpy()); xms.append(xm.cpu().numpy())
    h.destroy(); hm.destroy()
    return xs, xms


def test_results_identical_alone_and_in_the_mix(scr, systems):
    ctx = scr.Context(0)
    alone = [_alone(scr, ctx, sd) for sd in systems]
    srv = scr.Server(ctx, max_slots=3)
    ids, outs = [], []
    for rep in range(2):                      # every system twice: more requests than slots
        for sd in systems:
            xs = [torch.full_like(b, np.nan) for b in sd["b"]]
            xms = [torch.full_like(b, np.nan) for b in sd["bm"]]
            ids.append(srv.submit(sd["K"], sd["coords"], sd["b"], xs, L=sd["L"], bms=sd["bm"], xms=xms))
            outs.append((xs, xms))
    res = [srv.wait(i) for i in ids]
    max_active = srv.drain()
    torch.cuda.synchronize()
    for k, (r, (xs, xms)) in enumerate(zip(res, outs)):
        xa, xma = alone[k % len(systems)]
        assert r["status"] == 0, r
        assert r["n_solves"] == len(xs)
        assert r["latency_ms"] >= r["queue_ms"] >= 0
        for x, ref in zip(xs, xa):
            assert np.array_equal(x.cpu().numpy(), ref)
        for x, ref in zip(xms, xma):
            assert np.array_equal(x.cpu().numpy(), ref)
        # the served results solve their systems (the oracle's SpMV), and the request's measured peak
        # of device memory stays within the footprint it was admitted with
        sd = systems[k % len(systems)]
        s = sd["sys"]
        for x, b in zip(xs, sd["b"]):
            bh = b.cpu().numpy()
            res = bh - oracle.bsr_spmv(s.rp, s.ci, s.val, x.cpu().numpy())
            assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(bh), k
        for x, b in zip(xms, sd["bm"]):
            xh, bh = x.cpu().numpy(), b.cpu().numpy()
            for c in range(3):
                rc_ = bh[c::3] - oracle.bsr_spmv(s.Lrp, s.Lci, s.Lval, xh[c::3])
                assert np.linalg.norm(rc_) <= 1e-8 * max(np.linalg.norm(bh[c::3]), 1e-300), (k, c)
        print(f"[gpu] request {k}: n_b={sd['nb']} peak {r['device_bytes']} footprint {r['footprint']}", flush=True)
        assert 0 < r["device_bytes"] <= r["footprint"], (k, r["device_bytes"], r["footprint"])
    assert max_active >= 2                     # requests really overlapped
    srv.destroy()
    assert ctx.bytes_in_use() == 0
    ctx.destroy()


def test_admission_by_footprint_and_rejection(scr, systems):
    ctx = scr.Context(0)
    big = systems[4]
    fp = scr.footprint_estimate(scr.SCR_SYSTEM, big["nb"], big["K"][1].numel()) + \
        scr.footprint_estimate(scr.MESH_SYSTEM, big["nphys"], big["L"][1].numel())
    # room for one large request at a time: three of them must run one after the other
    srv = scr.Server(ctx, max_slots=3, hbm_budget=int(fp * 1.5))
    ids = []
    for _ in range(3):
        xs = [torch.zeros_like(b) for b in big["b"]]
        xms = [torch.zeros_like(b) for b in big["bm"]]
        ids.append(srv.submit(big["K"], big["coords"], big["b"], xs, L=big["L"], bms=big["bm"], xms=xms))
    res = [srv.wait(i) for i in ids]
    assert all(r["status"] == 0 for r in res)
    assert srv.drain() == 1
    assert res[2]["queue_ms"] > 0
    srv.destroy()
    # a request larger than the budget is rejected at submission, never queued
    srv = scr.Server(ctx, max_slots=2, hbm_budget=int(fp * 0.5))
    with pytest.raises(scr.ScrError) as e:
        srv.submit(big["K"], big["coords"], big["b"], [torch.zeros_like(b) for b in big["b"]])
    assert e.value.status == scr.SCR_E_OOM
    srv.destroy()
    ctx.destroy()


def test_failing_request_is_isolated(scr, systems):
    ctx = scr.Context(0)
    srv = scr.Server(ctx, max_slots=2)
    good = systems[1]
    bad_ci = good["K"][1].clone()
    bad_ci[[3, 4]] = bad_ci[[4, 3]]            # unsorted columns
    xg = [torch.zeros_like(b) for b in good["b"]]
    xb = [torch.zeros_like(b) for b in good["b"]]
    i_bad = srv.submit((good["K"][0], bad_ci, good["K"][2]), good["coords"], good["b"], xb)
    i_good = srv.submit(good["K"], good["coords"], good["b"], xg)
    rb, rg = srv.wait(i_bad), srv.wait(i_good)
    assert rb["status"] == scr.SCR_E_INVALID
    assert rg["status"] == 0
    xa, _ = _alone(scr, ctx, good)
    assert np.array_equal(xg[0].cpu().numpy(), xa[0])
    srv.destroy()
    assert ctx.bytes_in_use() == 0
    ctx.destroy()


def test_new_tangent_per_correction_matches_sequential_re_setups(scr):
    # three corrections whose tangents change (dt = 1e-3, 2e-3, 4e-3 on one mesh): the server's
    # numeric re-setups give bitwise what setup -> solve -> amg_update -> solve on one handle gives
    p = synth.cfg0_params()
    mats = []
    for dt in (1e-3, 2e-3, 4e-3):
        p.dt = dt
        mats.append(synth.generate(p))
    s0 = mats[0]
    assert all(np.array_equal(m.rp, s0.rp) and np.array_equal(m.ci, s0.ci) for m in mats)
    K = (dev(s0.rp), dev(s0.ci), dev(s0.val.reshape(-1)))
    coords = dev(s0.xyz.reshape(-1))
    bs = [dev(synth.rhs(700 + c, 4 * s0.n_b, s0.mask)) for c in range(3)]
    ctx = scr.Context(0)
    h = scr.amg_setup(ctx, scr.SCR_SYSTEM, *K, coords)
    ref = []
    for c in range(3):
        if c:
            scr.amg_update(h, K[0], K[1], dev(mats[c].val.reshape(-1)))
        x = torch.zeros_like(bs[c])
        rc, _ = scr.scr_solve(h, bs[c], x)
        assert rc == 0
        ref.append(x.cpu().numpy())
    h.destroy()
    srv = scr.Server(ctx, max_slots=2)
    xs = [torch.full_like(b, np.nan) for b in bs]
    xf = [torch.full_like(b, np.nan) for b in bs]
    i_new = srv.submit(K, coords, bs, xs, vals=[None] + [dev(m.val.reshape(-1)) for m in mats[1:]])
    i_frozen = srv.submit(K, coords, bs, xf)
    rn, rf = srv.wait(i_new), srv.wait(i_frozen)
    assert rn["status"] == 0 and rf["status"] == 0 and rn["n_solves"] == 3
    for c in range(3):
        assert np.array_equal(xs[c].cpu().numpy(), ref[c])
    assert np.array_equal(xf[0].cpu().numpy(), ref[0])
    assert not np.array_equal(xf[2].cpu().numpy(), ref[2])      # the frozen tangent is another system
    srv.destroy()
    assert ctx.bytes_in_use() == 0
    ctx.destroy()


def test_tangents_assembled_per_correction_match_sequential(scr):
    # three corrections at advective states 0, u and 2u (tangents assembled on the device from the
    # mesh): the server gives bitwise what assemble -> setup -> solve -> assemble -> amg_update ->
    # solve on one handle gives; a request with a frozen tangent runs beside it
    from oracle import assembly as asm
    p = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0, u_max=20.0)
    s = synth.generate(p, tets=True)
    ctx = scr.Context(0)
    a = scr.scr_assembler_create(ctx, dev(s.tv), dev(s.tp), dev(s.tsolid), dev(s.rp), dev(s.ci),
                                 dev(s.xyz.reshape(-1)), dev(s.mask), scr.tangent_params(**asm.params_of(p)))
    us = [None, dev(s.uadv), dev(2.0 * s.uadv)]
    K = (dev(s.rp), dev(s.ci), dev(s.val.reshape(-1)))
    coords = dev(s.xyz.reshape(-1))
    bs = [dev(synth.rhs(800 + c, 4 * s.n_b, s.mask)) for c in range(3)]
    ref, h = [], None
    for c in range(3):
        val = torch.empty(16 * a.nnzb, dtype=torch.float64, device="cuda")
        scr.scr_assemble_tangent(a, us[c], val)
        if c == 0:
            h = scr.amg_setup(ctx, scr.SCR_SYSTEM, K[0], K[1], val, coords)
        else:
            scr.amg_update(h, K[0], K[1], val)
        x = torch.zeros_like(bs[c])
        rc, _ = scr.scr_solve(h, bs[c], x)
        assert rc == 0
        ref.append(x.cpu().numpy())
    h.destroy()
    srv = scr.Server(ctx, max_slots=2)
    xs = [torch.full_like(b, np.nan) for b in bs]
    xf = [torch.full_like(b, np.nan) for b in bs]
    i_asm = srv.submit(K, coords, bs, xs, tangent=a, us=us)
    i_frozen = srv.submit(K, coords, bs, xf)
    ra, rf = srv.wait(i_asm), srv.wait(i_frozen)
    assert ra["status"] == 0 and rf["status"] == 0 and ra["n_solves"] == 3
    for c in range(3):
        assert np.array_equal(xs[c].cpu().numpy(), ref[c])
    assert not np.array_equal(xf[2].cpu().numpy(), ref[2])      # the frozen tangent is another system
    # an assembler on another pattern is rejected at submission
    p2 = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=6, R=1.0, L=2.0)
    s2 = synth.generate(p2, tets=True)
    a2 = scr.scr_assembler_create(ctx, dev(s2.tv), dev(s2.tp), dev(s2.tsolid), dev(s2.rp), dev(s2.ci),
                                  dev(s2.xyz.reshape(-1)), dev(s2.mask), scr.tangent_params(**asm.params_of(p2)))
    with pytest.raises(scr.ScrError) as e:
        srv.submit(K, coords, bs, xs, tangent=a2)
    assert e.value.status == scr.SCR_E_INVALID
    srv.destroy()
    a.destroy(); a2.destroy()
    assert ctx.bytes_in_use() == 0
    ctx.destroy()
