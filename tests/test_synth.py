"""Pins of the seeded input generator against closed forms and invariants of the paper's
discretisation (Sec. 3): generalized-alpha constants, P1 stiffness on the Kuhn grid, the metric
tensor's vertex-permutation invariance, rigid-motion kernels of the deviatoric operator, the
block structure [A G; D C] with D = -G^T, interface pressure duplication, Dirichlet rows."""
import itertools

import numpy as np
import pytest

import synth
from tests.conftest import bsr_to_dense


def test_genalpha_constants():
    # Sec. 3.4: alpha_m = (3 - rho)/(2(1 + rho)), alpha_f = gamma = 1/(1 + rho); rho = 0.5
    am, af, g = synth.genalpha(0.5)
    assert am == pytest.approx(5.0 / 6.0, abs=1e-15)
    assert af == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert g == pytest.approx(2.0 / 3.0, abs=1e-15)
    am, af, g = synth.genalpha(1.0)          # rho_inf = 1: trapezoidal (1/2, 1/2, 1/2)
    assert (am, af, g) == (0.5, 0.5, 0.5)


def _box(nx, ny, nz, h, **kw):
    p = synth.default_params(mode=1, m_core=nx, n_bl=ny, n_wall=0, nz=nz, R=h, **kw)
    return synth.generate(p, tets=True)


def test_box_stiffness_is_seven_point_stencil():
    # P1 on the Kuhn triangulation of a uniform grid reproduces the 7-point Laplacian:
    # stiffness = h * [6 on the diagonal, -1 on the six axis neighbours, 0 elsewhere].
    # The C block of the fluid is tau_M * stiffness (all Kuhn tets are congruent, one tau_M).
    h = 0.25
    s = _box(4, 4, 4, h, terms=16, apply_bc=0)
    C = bsr_to_dense(s.rp, s.ci, s.val[:, 3:4, 3:4])
    nx = ny = nz = 5
    idx = lambda i, j, k: i + nx * (j + ny * k)
    tauM = C[idx(2, 2, 2), idx(2, 2, 2)] / (6 * h)
    for (i, j, k) in [(1, 1, 1), (2, 2, 2), (3, 2, 1), (1, 3, 3)]:
        row = C[idx(i, j, k)] / (tauM * h)
        expect = np.zeros_like(row)
        expect[idx(i, j, k)] = 6.0
        for d in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
            expect[idx(i + d[0], j + d[1], k + d[2])] = -1.0
        assert np.abs(row - expect).max() < 1e-12


def test_mesh_laplacian_dirichlet_eigenvalues_closed_form():
    # L_ab = sum over elements of grad N_a . grad N_b (element factor 1/V).  On the uniform Kuhn
    # grid this is (6/h^2) * 7-point stencil; with Dirichlet on the boundary its interior
    # eigenvalues are (6/h^2) * sum_d 4 sin^2(k_d pi / (2 (n_d + 1))).
    h = 0.5
    nx, ny, nz = 5, 4, 3                       # cells
    s = _box(nx, ny, nz, h)
    L = bsr_to_dense(s.Lrp, s.Lci, s.Lval)
    interior = np.where(s.Lmask == 0)[0]
    ev = np.sort(np.linalg.eigvalsh(L[np.ix_(interior, interior)]))
    n = [nx - 1, ny - 1, nz - 1]
    closed = sorted((6 / h**2) * sum(4 * np.sin(k[d] * np.pi / (2 * (n[d] + 1)))**2 for d in range(3))
                    for k in itertools.product(*[range(1, n[d] + 1) for d in range(3)]))
    assert np.allclose(ev, closed, rtol=1e-12, atol=1e-12)
    # Dirichlet rows are identity rows with zeroed columns
    bnd = np.where(s.Lmask)[0]
    assert np.array_equal(L[np.ix_(bnd, bnd)], np.eye(bnd.size))
    assert not L[np.ix_(bnd, interior)].any() and not L[np.ix_(interior, bnd)].any()


def test_box_volume_and_mass():
    # sum of element volumes = box volume; consistent mass row sums = lumped volume
    h = 0.3
    s = _box(3, 2, 4, h, terms=1, apply_bc=0)
    p = synth.default_params()
    am, af, g = synth.genalpha(p.rho_inf)
    ct = am / (af * g * p.dt)
    A = bsr_to_dense(s.rp, s.ci, s.val[:, :3, :3])
    total = A.sum() / (3 * p.rho_f * ct)      # mass entries sum to the volume per component
    assert total == pytest.approx(3 * 2 * 4 * h**3, rel=1e-13)


def _random_tet(rng):
    while True:
        x = rng.normal(size=(4, 3))
        if abs(np.linalg.det(x[1:] - x[0])) > 0.2:
            return x


def test_tau_metric_is_vertex_permutation_invariant():
    # The regular-simplex matrix M makes G = J^-T M J^-1 independent of the vertex order (Sec. 3.2).
    rng = np.random.default_rng(3)
    p = synth.default_params()
    for _ in range(5):
        x = _random_tet(rng)
        vals = np.array([synth.tau(x[list(perm)], p) for perm in itertools.permutations(range(4))])
        assert np.ptp(vals[:, 0]) <= 1e-13 * vals[0, 0]
        assert np.ptp(vals[:, 1]) <= 1e-12 * vals[0, 1]


def test_tau_M_without_viscosity_is_dt_over_two_rho():
    # tau_M = rho^-1 (C_T/dt^2 + ...)^-1/2 with C_T = 4 and mu = 0 reduces to dt / (2 rho).
    p = synth.default_params(mu_f=0.0)
    x = _random_tet(np.random.default_rng(1))
    tm, _ = synth.tau(x, p)
    assert tm == pytest.approx(p.dt / (2 * p.rho_f), rel=1e-14)


def _rigid(x4):
    x = x4 - x4.mean(0)
    modes = []
    for c in range(3):
        m = np.zeros((4, 4)); m[:, c] = 1.0; modes.append(m)
    for (i, j) in [(0, 1), (1, 2), (2, 0)]:
        m = np.zeros((4, 4)); m[:, i] = -x[:, j]; m[:, j] = x[:, i]; modes.append(m)
    return [m.reshape(16) for m in modes]


@pytest.mark.parametrize("solid", [False, True])
def test_deviatoric_and_graddiv_annihilate_rigid_motions(solid):
    rng = np.random.default_rng(7)
    x = _random_tet(rng)
    for terms in (2, 4) if not solid else (2,):
        Ke, V = synth.element(x, synth.default_params(terms=terms), solid)
        vel = np.array([4 * a + i for a in range(4) for i in range(3)])
        for m in _rigid(x):
            assert np.abs(Ke @ m).max() <= 1e-10 * np.abs(Ke).max()
        Av = Ke[np.ix_(vel, vel)]
        assert np.allclose(Av, Av.T, atol=1e-12 * np.abs(Av).max())
    # grad-div is rank one (outer product of the divergence row)
    Ke, _ = synth.element(x, synth.default_params(terms=4), False)
    sv = np.linalg.svd(Ke, compute_uv=False)
    assert sv[1] <= 1e-12 * sv[0]


def test_element_G_D_C_structure():
    rng = np.random.default_rng(11)
    x = _random_tet(rng)
    p = synth.default_params()
    for solid in (False, True):
        Ke, V = synth.element(x, p, solid)
        vel = [4 * a + i for a in range(4) for i in range(3)]
        pre = [4 * a + 3 for a in range(4)]
        G = Ke[np.ix_(vel, pre)]
        D = Ke[np.ix_(pre, vel)]
        assert np.array_equal(D, -G.T)                       # D = -G^T exactly
        assert np.abs(G.reshape(4, 3, 4).sum(0)).max() < 1e-14  # sum_a dN_a = 0
        Cb = Ke[np.ix_(pre, pre)]
        assert np.allclose(Cb, Cb.T) and np.linalg.eigvalsh(Cb).min() > -1e-14 * np.abs(Cb).max()
        if solid:
            am, af, g = synth.genalpha(p.rho_inf)
            ct = am / (af * g * p.dt)
            kappa = p.E_s / (3 * (1 - 2 * p.nu_s))
            assert Cb.sum() == pytest.approx(ct / kappa * V, rel=1e-13)   # (c_t/kappa) * mass


def _pattern_bruteforce(s):
    pairs = set()
    for e in range(s.n_tets):
        va, pa = s.tv[e], s.tp[e]
        for a in range(4):
            for b in range(4):
                pairs.update({(va[a], va[b]), (va[a], pa[b]), (pa[a], va[b]), (pa[a], pa[b])})
    pairs.update((i, i) for i in range(s.n_b))
    return pairs


def test_K_pattern_matches_element_connectivity(tiny):
    got = {(i, int(c)) for i in range(tiny.n_b) for c in tiny.ci[tiny.rp[i]:tiny.rp[i + 1]]}
    assert got == _pattern_bruteforce(tiny)
    assert all(np.all(np.diff(tiny.ci[tiny.rp[i]:tiny.rp[i + 1]]) > 0) for i in range(tiny.n_b))


def test_cfg0_counts(cfg0):
    assert cfg0.n_phys == 13 * 13 * 41 == cfg0.n_b
    assert cfg0.n_tets == 6 * 12 * 12 * 40
    assert cfg0.nnzb == 94321
    dirichlet_nodes = int((cfg0.mask.reshape(-1, 4)[:, 0] > 0).sum())
    assert dirichlet_nodes == 48 * 41 + 11 * 11     # wall shell (48 nodes x 41 layers) + inlet interior
    assert not cfg0.mask.reshape(-1, 4)[:, 3].any()  # no pressure Dirichlet
    assert np.all(cfg0.kind == 0)


def test_block_structure_and_dirichlet(small_fsi):
    s = small_fsi
    nb = s.n_b
    Kd = bsr_to_dense(s.rp, s.ci, s.val)
    vel = np.array([4 * i + c for i in range(nb) for c in range(3)])
    pre = np.arange(nb) * 4 + 3
    A = Kd[np.ix_(vel, vel)]; G = Kd[np.ix_(vel, pre)]; D = Kd[np.ix_(pre, vel)]; Cb = Kd[np.ix_(pre, pre)]
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    assert np.array_equal(D, -G.T)
    assert np.allclose(Cb, Cb.T, atol=1e-14 * np.abs(Cb).max())
    # Dirichlet dofs: identity row and zero column
    dd = np.where(s.mask)[0]
    for d in dd[:200]:
        row = Kd[d].copy(); col = Kd[:, d].copy()
        assert row[d] == 1.0 and col[d] == 1.0
        row[d] = 0; col[d] = 0
        assert not row.any() and not col.any()
    # interface duplication: one virtual block row per interface node, velocity slots Dirichlet
    virt = np.where(s.kind == 3)[0]
    assert virt.size == s.n_iface == np.sum(s.kind == 2)
    assert np.all(virt - 1 == np.where(s.kind == 2)[0])      # virtual row right after its node
    assert np.all(s.mask.reshape(-1, 4)[virt, :3] == 1)
    # solid elements use the virtual node's pressure, fluid elements the physical one
    virt_set = set(virt.tolist())
    for e in range(s.n_tets):
        uses_virtual = any(int(q) in virt_set for q in s.tp[e])
        if uses_virtual:
            assert s.tsolid[e] == 1
        if not s.tsolid[e]:
            assert np.array_equal(s.tp[e], s.tv[e])
    # the Schur-like pressure operator C + G^T diag(A)^-1 G is SPD (A SPD)
    free = np.where(s.mask.reshape(-1, 4)[:, :3].reshape(-1) == 0)[0]
    assert np.linalg.eigvalsh(A[np.ix_(free, free)]).min() > 0


def test_positive_volumes_and_conformity(small_fsi):
    s = small_fsi
    x = s.xyz
    vols = []
    for e in range(s.n_tets):
        v = x[s.tv[e]]
        vols.append(np.linalg.det(v[1:] - v[0]) / 6)
    vols = np.array(vols)
    assert vols.min() > 0
    # faces are shared by at most two tets (conforming triangulation)
    faces = {}
    for e in range(s.n_tets):
        for f in itertools.combinations(sorted(s.tv[e].tolist()), 3):
            faces[f] = faces.get(f, 0) + 1
    assert max(faces.values()) == 2


def test_rhs_determinism_and_range():
    mask = np.zeros(1000, np.uint8); mask[::7] = 1
    a = synth.rhs(5, 1000, mask); b = synth.rhs(5, 1000, mask); c = synth.rhs(6, 1000, mask)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.all(a[mask == 1] == 0) and a.min() >= -1 and a.max() < 1
    assert abs(a[mask == 0].mean()) < 0.1


# ---------------------------------------------------------------- Y-bifurcation (voxel) workload
def _branches(p):
    """(start, unit direction, length, radius, cap at far end) of the three branches, written
    from the workload's definition (parent along +z into the junction at the origin, daughters
    leaving it in the x-z plane)."""
    t1, t2 = p.y_th1, p.y_th2
    return [(np.array([0.0, 0.0, -p.L]), np.array([0.0, 0.0, 1.0]), p.L, p.R, True),
            (np.zeros(3), np.array([np.sin(t1), 0.0, np.cos(t1)]), p.y_ld, p.y_rd * p.R, False),
            (np.zeros(3), np.array([-np.sin(t2), 0.0, np.cos(t2)]), p.y_ld, p.y_rd * p.R, False)]


def _rel_dist(p, x):
    """min over branches of distance / radius (inf beyond a free-end cut), points x (n, 3)."""
    best = np.full(len(x), np.inf)
    for a, u, ln, r, cap_end in _branches(p):
        d = x - a
        t = d @ u
        radial = np.linalg.norm(d - t[:, None] * u, axis=1)
        junction = np.linalg.norm(d - (ln if cap_end else 0.0) * u, axis=1)
        beyond_free = t < 0 if cap_end else t > ln
        in_cap = t > ln if cap_end else t < 0
        dist = np.where(in_cap, junction, radial) / r
        dist[beyond_free] = np.inf
        best = np.minimum(best, dist)
    return best


@pytest.fixture(scope="module")
def ysmall():
    p = synth.y_params(h=0.25, seed=3)
    return p, synth.generate(p, tets=True)


def test_y_angles_seeded_in_range():
    for seed in range(5):
        p = synth.y_params(h=0.5, seed=seed)
        for th in (p.y_th1, p.y_th2):
            assert np.deg2rad(30) <= th <= np.deg2rad(60)
    assert synth.y_params(h=0.5, seed=1).y_th1 == synth.y_params(h=0.5, seed=1).y_th1
    assert synth.y_params(h=0.5, seed=1).y_th1 != synth.y_params(h=0.5, seed=2).y_th1


def test_y_voxels_tets_and_classification(ysmall):
    p, s = ysmall
    x = s.xyz
    h = p.y_h
    # every vertex on the voxel grid with the inlet plane z = -L as a grid plane
    assert np.allclose((x[:, 2] + p.L) / h, np.round((x[:, 2] + p.L) / h), atol=1e-9)
    # six congruent Kuhn tets per kept voxel, all positively oriented with volume h^3/6
    v = x[s.tv]
    vol = np.einsum("ij,ij->i", np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), v[:, 3] - v[:, 0]) / 6
    assert s.n_tets % 6 == 0 and np.allclose(vol, h ** 3 / 6, rtol=1e-9)
    # voxels kept: centre inside the wall region (relative distance < 1.2); tets fluid iff the
    # centroid is inside the lumen (relative distance < 1)
    cen = v.mean(axis=1)
    rel = _rel_dist(p, cen)
    assert np.array_equal(s.tsolid == 0, rel < 1.0)
    vox = (v.min(axis=1) + v.max(axis=1)) / 2
    assert np.all(_rel_dist(p, vox) < p.wall_ratio)
    # conforming: every face shared by at most two tets
    faces = np.sort(np.concatenate([s.tv[:, [0, 1, 2]], s.tv[:, [0, 1, 3]], s.tv[:, [0, 2, 3]],
                                    s.tv[:, [1, 2, 3]]]), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert counts.max() == 2


def test_y_block_structure_interface_and_dirichlet(ysmall):
    import scipy.sparse as sp
    p, s = ysmall
    nb = s.n_b
    K = sp.bsr_matrix((s.val, s.ci, s.rp), shape=(4 * nb, 4 * nb)).tocsr()
    K.eliminate_zeros()
    vel = (np.arange(nb)[:, None] * 4 + np.arange(3)).reshape(-1)
    pre = np.arange(nb) * 4 + 3
    A = K[vel][:, vel]; G = K[vel][:, pre]; D = K[pre][:, vel]; Cb = K[pre][:, pre]
    amax = abs(A).max()
    assert abs(A - A.T).max() <= 1e-12 * amax
    assert abs(D + G.T).max() == 0
    assert abs(Cb - Cb.T).max() <= 1e-14 * abs(Cb).max()
    # interface: nodes touching both fluid and solid tets, each followed by its virtual node
    kind = s.kind
    touch = np.zeros(nb, np.uint8)
    np.bitwise_or.at(touch, s.tv[s.tsolid == 0].reshape(-1), 1)
    np.bitwise_or.at(touch, s.tv[s.tsolid == 1].reshape(-1), 2)
    phys = kind != 3
    assert np.array_equal(kind[phys] == 2, touch[phys] == 3)
    assert np.array_equal(kind[phys] == 0, touch[phys] == 1)
    virt = np.where(kind == 3)[0]
    assert np.array_equal(virt - 1, np.where(kind == 2)[0]) and virt.size == s.n_iface
    # solid tets take pressure from the virtual node of interface vertices
    solid_tp = s.tp[s.tsolid == 1]
    assert np.all(np.isin(solid_tp[kind[s.tv[s.tsolid == 1]] == 2],
                          virt)) and np.array_equal(s.tp[s.tsolid == 0], s.tv[s.tsolid == 0])
    # Dirichlet velocity: the whole inlet plane, identity rows and zero columns
    m = s.mask.reshape(-1, 4)
    inlet = np.isclose(s.xyz[:, 2], -p.L) & phys
    assert np.all(m[inlet, :3] == 1) and not m[:, 3].any()
    d = np.where(s.mask)[0]
    Kd = K[d]
    assert np.array_equal(Kd.indices, d) and np.all(Kd.data == 1.0)
    assert abs(K[:, d]).sum() == d.size
    # the fluid part of the outlets stays free (traction-free); the solid ends are clamped
    assert np.all(m[(kind == 0) & ~inlet, :3] == 0)


def test_y_mesh_laplacian(ysmall):
    import scipy.sparse as sp
    p, s = ysmall
    L = sp.csr_matrix((s.Lval, s.Lci, s.Lrp), shape=(s.n_phys, s.n_phys))
    assert abs(L - L.T).max() <= 1e-13 * abs(L).max()
    # every node not strictly inside the lumen is Dirichlet (identity row and column)
    solid_nodes = np.zeros(s.n_b, bool)
    solid_nodes[s.tv[s.tsolid == 1].reshape(-1)] = True
    bop = s.blk_of_phys
    assert np.all(s.Lmask[solid_nodes[bop]] == 1)
    free = np.where(s.Lmask == 0)[0]
    # P1 stiffness annihilates constants: interior free rows sum to zero where no Dirichlet
    # neighbour was eliminated
    Lf = L[free]
    pat = sp.csr_matrix((np.ones(s.Lci.size), s.Lci, s.Lrp), shape=L.shape)   # stored pattern
    nbr_dir = np.asarray(pat[free][:, np.where(s.Lmask == 1)[0]].sum(axis=1)).ravel()
    full = nbr_dir == 0
    raw = np.asarray(Lf.sum(axis=1)).ravel()
    assert full.any() and np.abs(raw[full]).max() <= 1e-12 * abs(L).max()


# ----------------------------------------------------------------------------- advective state and outlets
def _bary_grad(x4):
    """Gradients of the barycentric coordinates of a tetrahedron (rows), from the 4x4 system
    [1 x y z] lambda = e (independent of the generator's Jacobian inverse)."""
    T = np.hstack([np.ones((4, 1)), x4])
    return np.linalg.inv(T)[1:].T            # (4, 3): grad lambda_a


def test_reaction_term_alone_for_a_linear_field_with_zero_centroid_velocity():
    # u(x) = B (x - centroid): the centroid velocity is zero, so tau_M and every advective term
    # vanish except the reaction rho * M_ab * grad u with grad u = B (P1 is exact on linear fields)
    rng = np.random.default_rng(21)
    x = _random_tet(rng)
    B = rng.normal(size=(3, 3))
    u4 = (x - x.mean(0)) @ B.T
    p = synth.default_params()
    K0, V = synth.element(x, p, False)
    K1, _ = synth.element(x, p, False, u4)
    dK = (K1 - K0).reshape(4, 4, 4, 4)        # [a, c, b, d]
    M = V * (np.ones((4, 4)) + np.eye(4)) / 20.0
    expect = p.rho_f * M[:, None, :, None] * np.pad(B, ((0, 1), (0, 1)))[None, :, None, :]
    assert np.abs(dK - expect).max() <= 1e-13 * np.abs(K1).max()


def test_uniform_advection_terms_match_quadrature_of_the_weak_form():
    # uniform u, only the advection bit: the element integrals of the Oseen VMS terms, evaluated
    # by a degree-2 quadrature with independently computed shape functions
    rng = np.random.default_rng(22)
    x = _random_tet(rng)
    u = rng.normal(size=3)
    p = synth.default_params(terms=32)
    Ke, V = synth.element(x, p, False, np.tile(u, (4, 1)))
    tauM, _ = synth.tau(x, p, u)
    am, af, g = synth.genalpha(p.rho_inf)
    ct = am / (af * g * p.dt)
    rho = p.rho_f
    dN = _bary_grad(x)
    a_, b_ = 0.5854101966249685, 0.1381966011250105
    pts = [np.roll([a_, b_, b_, b_], k) for k in range(4)]            # barycentric points, weight V/4
    ud = dN @ u                                                        # u . grad N_a
    A = np.zeros((4, 4)); G = np.zeros((4, 3, 4)); D = np.zeros((4, 4, 3))
    for lam in pts:
        w = V / 4.0
        A += w * (rho * np.outer(lam, ud) + tauM * rho * rho * np.outer(ud, ct * lam + ud))
        G += w * tauM * rho * ud[:, None, None] * dN.T[None, :, :]
        D += w * tauM * rho * dN[:, None, :] * ud[None, :, None]
    K = Ke.reshape(4, 4, 4, 4)
    scale = np.abs(Ke).max()
    for i in range(3):
        for j in range(3):
            assert np.abs(K[:, i, :, j] - (A if i == j else 0.0)).max() <= 1e-12 * scale
        assert np.abs(K[:, i, :, 3] - G[:, i, :]).max() <= 1e-12 * scale
        assert np.abs(K[:, 3, :, i] - D[:, :, i]).max() <= 1e-12 * scale
    assert np.abs(K[:, 3, :, 3]).max() == 0.0


def test_tau_M_with_advection_and_no_viscosity():
    # mu = 0: tau_M = rho^-1 (4/dt^2 + u.G.u)^-1/2; for a velocity field along one edge direction
    # the metric term is positive and tau_M falls below dt/(2 rho)
    p = synth.default_params(mu_f=0.0)
    x = _random_tet(np.random.default_rng(23))
    t0, _ = synth.tau(x, p, np.zeros(3))
    assert t0 == pytest.approx(p.dt / (2 * p.rho_f), rel=1e-14)
    u = 50.0 * (x[1] - x[0])
    t1, _ = synth.tau(x, p, u)
    uGu = (1.0 / (p.rho_f * t1)) ** 2 - 4.0 / p.dt ** 2
    assert t1 < t0 and uGu > 0.0
    t2, _ = synth.tau(x, p, 2.0 * u)                  # u.G.u is quadratic in u
    assert (1.0 / (p.rho_f * t2)) ** 2 - 4.0 / p.dt ** 2 == pytest.approx(4.0 * uGu, rel=1e-9)


def test_advective_state_and_nonsymmetric_velocity_block(small_fsi_flow):
    import scipy.sparse as sp
    s0, s1 = small_fsi_flow
    assert np.array_equal(s0.rp, s1.rp) and np.array_equal(s0.ci, s1.ci)
    fluid = np.isin(s1.kind, (0, 2))
    r = np.hypot(s1.xyz[:, 0], s1.xyz[:, 1])
    expect = np.where(fluid, 30.0 * np.clip(1.0 - r ** 2, 0.0, None), 0.0)
    assert np.allclose(s1.uadv[:, 2], expect, rtol=0, atol=1e-12) and not s1.uadv[:, :2].any()
    A = lambda s: bsr_to_dense(s.rp, s.ci, s.val[:, :3, :3])
    A0, A1 = A(s0), A(s1)
    assert np.abs(A0 - A0.T).max() <= 1e-13 * np.abs(A0).max()
    assert np.abs(A1 - A1.T).max() > 1e-3 * np.abs(A1).max()
    # rows and columns of purely solid nodes see no fluid element: unchanged
    solid_rows = np.repeat(s1.kind == 1, 3)
    assert np.array_equal(A0[solid_rows][:, solid_rows], A1[solid_rows][:, solid_rows])
    # the advective state makes every fluid element's contribution differ, but Dirichlet rows stay
    d = np.where(s1.mask)[0]
    K1 = sp.csr_matrix(bsr_to_dense(s1.rp, s1.ci, s1.val))
    assert np.all(K1[d].data == 1.0) and abs(K1[:, d]).sum() == d.size


@pytest.fixture(scope="module")
def small_fsi_flow():
    kw = dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)
    return synth.generate(synth.default_params(**kw)), synth.generate(synth.default_params(u_max=30.0, **kw))


def test_outlet_vector_is_the_outlet_face_area_distribution():
    # without Dirichlet elimination the weights are the P1 integrals of N_A over the outlet face:
    # they sum to the area of the regular 8*m-gon that bounds the lumen, and sit on z = L only
    kw = dict(mode=0, m_core=3, n_bl=1, n_wall=0, nz=4, R=1.0, L=2.0)
    s = synth.generate(synth.default_params(apply_bc=0, **kw))
    assert len(s.outlets) == 1
    blk, a = s.outlets[0]
    N = 8 * 4
    assert a[:, 2].sum() == pytest.approx(0.5 * N * np.sin(2 * np.pi / N), rel=1e-13)
    assert not a[:, :2].any() and np.all(a[:, 2] > 0)
    assert np.all(s.xyz[blk, 2] == s.xyz[:, 2].max())
    # each vertex of the regular triangulated disk gets a third of its incident triangle areas:
    # the centre node of the section touches 8 triangles of the innermost shell
    centre = np.where((np.hypot(s.xyz[blk, 0], s.xyz[blk, 1]) == 0.0))[0]
    assert centre.size == 1
    # with Dirichlet elimination the wall ring is dropped (no-slip) and the rest is unchanged
    s2 = synth.generate(synth.default_params(apply_bc=1, **kw))
    blk2, a2 = s2.outlets[0]
    keep = np.isin(blk, blk2)
    assert np.array_equal(blk[keep], blk2) and np.array_equal(a[keep], a2)
    ring = np.hypot(s.xyz[blk[~keep], 0], s.xyz[blk[~keep], 1])
    assert np.allclose(ring, 1.0, rtol=0, atol=1e-12) and ring.size == N
