import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def cfg0():
    import synth
    return synth.generate(synth.cfg0_params(), tets=True)


@pytest.fixture(scope="session")
def tiny():
    """Smallest fluid+solid system (5x5 section, 3 axial cells, interface virtual nodes)."""
    import synth
    return synth.generate(synth.tiny_annulus_params(), tets=True)


@pytest.fixture(scope="session")
def small_fsi():
    """A small unified tube (9x9 section: 2 core + 1 BL + 1 wall shells, 8 axial cells)."""
    import synth
    p = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)
    return synth.generate(p, tets=True)


def bsr_to_dense(rp, ci, val, ncols=None):
    rp = np.asarray(rp); ci = np.asarray(ci); val = np.asarray(val)
    if val.ndim == 1:
        val = val.reshape(-1, 1, 1)
    nr = rp.size - 1
    br, bc = val.shape[1], val.shape[2]
    nc = ncols if ncols is not None else (int(ci.max()) + 1 if ci.size else 0)
    M = np.zeros((nr * br, nc * bc))
    for i in range(nr):
        for q in range(rp[i], rp[i + 1]):
            M[i * br:(i + 1) * br, ci[q] * bc:(ci[q] + 1) * bc] += val[q]
    return M


def split_perm(nb):
    """Permutation taking interleaved [vx vy vz p] per node to split [v (3nb); p (nb)]."""
    v = np.arange(4 * nb).reshape(nb, 4)
    return np.concatenate([v[:, :3].reshape(-1), v[:, 3]])


def field_errors(x, xref):
    """Relative errors of the velocity and the pressure parts of node-interleaved [vx vy vz p]
    vectors, each against its own norm (the pressure dominates the norm of the whole vector)."""
    x4 = np.asarray(x).reshape(-1, 4)
    r4 = np.asarray(xref).reshape(-1, 4)
    ev = np.linalg.norm(x4[:, :3] - r4[:, :3]) / np.linalg.norm(r4[:, :3])
    ep = np.linalg.norm(x4[:, 3] - r4[:, 3]) / np.linalg.norm(r4[:, 3])
    return float(ev), float(ep)


def assert_fields(x, xref, tol, what=""):
    """Velocity and pressure each within tol of their own reference norms (printed first)."""
    ev, ep = field_errors(x, xref)
    print(f"[fields] {what} velocity err {ev:.2e}, pressure err {ep:.2e} (tol {tol:.0e})", flush=True)
    assert ev <= tol and ep <= tol, (what, ev, ep)
