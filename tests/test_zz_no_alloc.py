"""mesh_motion_solve_noalloc: the mesh-motion solve with its CG workspace in the library's static
device scratch instead of the handle's memory.  Through the C ABI: bitwise the result of
mesh_motion_solve on two calls in a row (the second on a smaller mesh), no growth of the handle's
or the context's device memory, and a clear error for a mesh larger than the scratch."""
import numpy as np
import pytest

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


def _mesh(scr, ctx, s, precision):
    return scr.amg_setup(ctx, scr.MESH_SYSTEM, dev(s.Lrp), dev(s.Lci), dev(s.Lval), None,
                         scr.amg_opts(precision=precision))


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_mesh_solve_matches_the_allocating_one(scr, precision):
    big = synth.generate(synth.cfg0_params())
    small = synth.generate(synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0))
    assert small.n_phys < big.n_phys
    ctx = scr.Context(0)
    so = scr.solve_opts(tol=1e-10, max_it=500)
    for k, s in enumerate((big, small)):       # two calls in a row, the second on the smaller mesh
        print(f"[gpu] noalloc call {k}: n={s.n_phys} precision={precision}", flush=True)
        b = dev(synth.rhs(40 + k, 3 * s.n_phys, np.repeat(s.Lmask, 3)))
        h = _mesh(scr, ctx, s, precision)
        held, in_use = h.bytes(), ctx.bytes_in_use()
        x0 = torch.full_like(b, np.nan)
        rc0, st0 = scr.mesh_motion_solve_noalloc(h, b, x0, so)
        assert h.bytes() == held and ctx.bytes_in_use() == in_use     # nothing allocated
        x1 = torch.full_like(b, np.nan)
        rc1, st1 = scr.mesh_motion_solve(h, b, x1, so)
        assert rc0 == 0 and rc1 == 0
        assert st0["mesh_its"] == st1["mesh_its"] and st0["mesh_rel"] == st1["mesh_rel"]
        assert np.array_equal(x0.cpu().numpy(), x1.cpu().numpy())
        # and again after the allocating call (the scratch keeps the last call's contents)
        x2 = torch.full_like(b, np.nan)
        rc2, _ = scr.mesh_motion_solve_noalloc(h, b, x2, so)
        assert rc2 == 0 and np.array_equal(x2.cpu().numpy(), x1.cpu().numpy())
        h.destroy()
    ctx.destroy()


def test_noalloc_rejects_a_mesh_larger_than_the_scratch(scr):
    # a chain Laplacian of 2.4M nodes: its CG workspace exceeds the 256 MiB scratch
    n = 2_400_000
    rp = np.zeros(n + 1, np.int64)
    deg = np.full(n, 3); deg[0] = deg[-1] = 2
    rp[1:] = np.cumsum(deg)
    ci = np.empty(rp[-1], np.int32); v = np.empty(rp[-1])
    i = np.arange(n)
    pos = rp[:-1].copy()
    for off, val in ((-1, -1.0), (0, 2.0), (1, -1.0)):
        j = i + off
        ok = (j >= 0) & (j < n)
        ci[pos[ok]] = j[ok]; v[pos[ok]] = val
        pos[ok] += 1
    v[rp[:-1][[0]]] = 3.0           # a Dirichlet-like end keeps L nonsingular
    ctx = scr.Context(0)
    h = scr.amg_setup(ctx, scr.MESH_SYSTEM, dev(rp.astype(np.int32)), dev(ci), dev(v))
    b = dev(np.ones(3 * n))
    x = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    with pytest.raises(scr.ScrError) as e:
        scr.mesh_motion_solve_noalloc(h, b, x)
    assert e.value.status == scr.SCR_E_INVALID and "scratch" in str(e.value)
    assert not x.cpu().numpy().any()
    h.destroy()
    ctx.destroy()
