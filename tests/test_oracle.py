"""Pins of the FP64 oracle against what the mathematics fixes: exact solutions of integer
systems, textbook special cases, invariants of maximal independent sets, aggregates and
Galerkin products, closed-form smoother polynomials, the minimal-residual property of GMRES,
the CG iteration bound, the block-LDU identity behind SCR (Sec. 5.2.1) and dense LU on tiny
systems.  Each check is chosen so that a dropped term, a wrong sign or a transposed operand in
the oracle fails it."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import bsr_to_dense, split_perm


# ----------------------------------------------------------------------------- dense LU
def test_dense_lu_recovers_integer_solution():
    rng = np.random.default_rng(0)
    n = 40
    A = rng.integers(-5, 6, size=(n, n)).astype(float)
    x = rng.integers(-9, 10, size=n).astype(float)
    b = A @ x                                   # exact in FP64 (small integers)
    assert np.abs(oracle.dense_solve(A, b) - x).max() < 1e-9
    Pm = np.eye(4)[[2, 0, 3, 1]]                # zero diagonal: needs pivoting
    assert np.allclose(oracle.dense_solve(Pm, np.array([1.0, 2, 3, 4])), Pm.T @ [1.0, 2, 3, 4])


# ----------------------------------------------------------------------------- helpers
def _laplacian_box(nx, ny, nz, bc=True):
    s = synth.generate(synth.default_params(mode=1, m_core=nx, n_bl=ny, nz=nz, R=1.0,
                                            apply_bc=int(bc)))
    return s.Lrp, s.Lci, s.Lval, s


def _graph(rp, ci, flags):
    n = rp.size - 1
    return [set(int(ci[q]) for q in range(rp[i], rp[i + 1]) if flags[q]) for i in range(n)]


def _ball2(adj, i):
    b = set(adj[i])
    for j in adj[i]:
        b |= adj[j]
    b.discard(i)
    return b


# ----------------------------------------------------------------------------- strength
def test_strength_scalar_reduces_to_classical_SA_criterion(cfg0):
    # for 1x1 blocks: f_ij^2 >= theta^4 f_ii f_jj  <=>  |a_ij| >= theta sqrt(|a_ii a_jj|)
    rp, ci, val, _ = _laplacian_box(5, 4, 4, bc=True)
    rng = np.random.default_rng(1)
    val = val * (1 + 0.3 * rng.random(val.size))       # break the stencil symmetry of values
    theta = 0.3
    flags, iso = oracle.strength(rp, ci, val, theta)
    d = np.array([val[rp[i] + np.searchsorted(ci[rp[i]:rp[i + 1]], i)] for i in range(rp.size - 1)])
    row = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    s1 = np.abs(val) >= theta * np.sqrt(np.abs(d[row] * d[ci]))
    # symmetrised by OR through the transposed entry
    M = {(int(r), int(c)): bool(v) for r, c, v in zip(row, ci, s1)}
    expect = np.array([(M[(r, c)] or M.get((c, r), False)) and r != c for r, c in zip(row, ci)])
    assert np.array_equal(flags.astype(bool), expect)
    has = np.zeros(rp.size - 1, bool); np.logical_or.at(has, row, expect)
    assert np.array_equal(iso.astype(bool), ~has)


def test_dirichlet_and_virtual_rows_are_isolated(small_fsi):
    o = oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz)
    rp, ci, A = o.matrix("A")
    flags, iso = oracle.strength(rp, ci, A, 0.08)
    vmask = small_fsi.mask.reshape(-1, 4)[:, 0] == 1
    assert np.all(iso[vmask] == 1)


# ----------------------------------------------------------------------------- MIS-2
def test_mis2_is_the_greedy_distance2_mis(cfg0):
    rp, ci, val, _ = _laplacian_box(6, 5, 5)
    for theta, seed, level in [(0.1, 0, 0), (0.1, 9, 2), (0.5, 3, 1)]:
        flags, iso = oracle.strength(rp, ci, val, theta)
        root = oracle.mis2(rp, ci, flags, iso, seed, level)
        adj = _graph(rp, ci, flags)
        key = {i: oracle.mis_key(seed, level, i) for i in range(rp.size - 1)}
        S = {i for i in range(rp.size - 1) if root[i]}
        assert not any(root[i] for i in np.where(iso)[0])
        for i in range(rp.size - 1):
            if iso[i]:
                continue
            ball = _ball2(adj, i)
            # independence in G^2 and maximality
            if i in S:
                assert not (ball & S)
            else:
                assert ball & S
            # greedy fixed point: i in S  <=>  no selected node of larger key within distance 2
            assert (i in S) == (not any(key[j] > key[i] for j in ball & S))


def test_mis_keys_unique_and_seeded():
    k0 = [oracle.mis_key(0, 0, i) for i in range(2000)]
    k1 = [oracle.mis_key(1, 0, i) for i in range(2000)]
    assert len(set(k0)) == 2000 and k0 != k1
    assert all((k & 0xFFFFFFFF) == i for i, k in enumerate(k0))


# ----------------------------------------------------------------------------- aggregation
def test_aggregates_partition_and_shape(cfg0):
    rp, ci, val, _ = _laplacian_box(7, 6, 5)
    flags, iso = oracle.strength(rp, ci, val, 0.1)
    root = oracle.mis2(rp, ci, flags, iso, 4, 0)
    na, agg = oracle.aggregate(rp, ci, flags, iso, root, 4, 0)
    adj = _graph(rp, ci, flags)
    assert na == root.sum()
    assert np.all(agg[iso == 1] == -1) and np.all(agg[iso == 0] >= 0)
    roots = np.where(root)[0]
    assert np.array_equal(agg[roots], np.arange(na))            # roots numbered ascending
    for i in np.where((iso == 0) & (root == 0))[0]:
        r = roots[agg[i]]
        if r in adj[i]:
            continue                                             # distance-1 member
        # distance-2 member: joined through a distance-1 member of the same aggregate
        mids = [j for j in adj[i] if roots[agg[j]] in adj[j] and not root[j]]
        assert mids
        best = max(mids, key=lambda j: oracle.mis_key(4, 0, j))
        assert agg[best] == agg[i]


# ----------------------------------------------------------------------------- hierarchy invariants
@pytest.fixture(scope="module")
def scr_small(small_fsi):
    return oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz,
                      oracle.amg_opts(coarse_max=60))


def test_tentative_prolongator_reproduces_near_null_space(scr_small):
    for h in (scr_small.amgA, scr_small.amgS):
        assert h.nlevels >= 2
        for l in range(h.nlevels - 1):
            i = h.info(l)
            b, k = i["b"], i["k"]
            Q = h.get(l, "Q"); B = h.get(l, "B"); agg = h.get(l, "agg")
            Bc = h.get(l + 1, "B").reshape(i["nagg"], k, k)
            dead = h.get(l, "dead").reshape(i["nagg"], k)
            rows = np.repeat(agg, b)
            for a in range(i["nagg"]):
                sel = np.where(rows == a)[0]
                Qa = Q[sel]
                alive = dead[a] == 0
                assert np.allclose(Qa[:, alive].T @ Qa[:, alive], np.eye(alive.sum()), atol=1e-12)
                assert not Qa[:, ~alive].any()
                R = Bc[a]
                assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) >= 0)
                assert np.allclose(Qa @ R, B[sel], atol=1e-9 * max(1, np.abs(B[sel]).max()))
            assert not Q[np.repeat(agg < 0, b)].any()


def test_smoothed_prolongator_and_galerkin_product_dense(scr_small):
    for h in (scr_small.amgA, scr_small.amgS):
        for l in range(h.nlevels - 1):
            i = h.info(l)
            b, k = i["b"], i["k"]
            A = bsr_to_dense(h.get(l, "A.rp"), h.get(l, "A.ci"), h.get(l, "A.v"), i["nr"])
            Dinv = np.zeros_like(A)
            for r in range(i["nr"]):
                blk = A[r * b:(r + 1) * b, r * b:(r + 1) * b]
                Dinv[r * b:(r + 1) * b, r * b:(r + 1) * b] = np.linalg.inv(blk)
            lam = np.abs(Dinv @ A).sum(1).max()
            assert i["lam"] == pytest.approx(lam, rel=1e-12)
            Ql = h.get(l, "Q")
            agg = h.get(l, "agg")
            Q = np.zeros((A.shape[0], i["nagg"] * k))
            for r in range(A.shape[0]):
                if agg[r // b] >= 0:
                    Q[r, agg[r // b] * k:(agg[r // b] + 1) * k] = Ql[r]
            Pd = (np.eye(A.shape[0]) - 4 / (3 * lam) * Dinv @ A) @ Q
            iso = np.repeat(agg < 0, b)
            Pd[iso] = 0.0
            P = bsr_to_dense(h.get(l, "P.rp"), h.get(l, "P.ci"), h.get(l, "P.v"), i["nagg"])
            assert np.abs(P - Pd).max() <= 1e-12 * np.abs(Pd).max()
            R = bsr_to_dense(h.get(l, "R.rp"), h.get(l, "R.ci"), h.get(l, "R.v"), i["nr"])
            assert np.array_equal(R, P.T)
            Ac = P.T @ A @ P
            dead = np.where(h.get(l, "dead"))[0]
            Ac[dead, dead] = 1.0
            j = h.info(l + 1)
            Acg = bsr_to_dense(h.get(l + 1, "A.rp"), h.get(l + 1, "A.ci"), h.get(l + 1, "A.v"), j["nr"])
            assert np.abs(Acg - Ac).max() <= 1e-11 * np.abs(Ac).max()
            assert np.abs(Acg - Acg.T).max() <= 1e-12 * np.abs(Acg).max()
            # structural pattern of P: aggregates of the non-isolated neighbours of aggregated rows
            prp, pci = h.get(l, "P.rp"), h.get(l, "P.ci")
            arp, aci, agg = h.get(l, "A.rp"), h.get(l, "A.ci"), h.get(l, "agg")
            for r in range(i["nr"]):
                exp = sorted({int(agg[c]) for c in aci[arp[r]:arp[r + 1]] if agg[c] >= 0}) if agg[r] >= 0 else []
                assert list(pci[prp[r]:prp[r + 1]]) == exp


def test_galerkin_neumann_laplacian_annihilates_coarse_constants():
    rp, ci, val, _ = _laplacian_box(6, 6, 6, bc=False)
    n = rp.size - 1
    h = oracle.Amg(rp, ci, val, np.ones((n, 1)), oracle.amg_opts(coarse_max=20, theta=0.05))
    assert h.nlevels >= 2
    for l in range(1, h.nlevels):
        i = h.info(l)
        Ac = bsr_to_dense(h.get(l, "A.rp"), h.get(l, "A.ci"), h.get(l, "A.v"), i["nr"])
        # P reproduces the constant (R(1) = 1 on every aggregate) so R A P 1_c = R A 1 = 0
        Bc = h.get(l, "B")
        assert np.abs(Ac @ Bc[:, 0]).max() <= 1e-12 * np.abs(Ac).max()


# ----------------------------------------------------------------------------- smoothers and V-cycle
def _dense_level(h, l):
    i = h.info(l)
    A = bsr_to_dense(h.get(l, "A.rp"), h.get(l, "A.ci"), h.get(l, "A.v"), i["nr"])
    Dinv = np.zeros_like(A)
    b = i["b"]
    Dv = h.get(l, "Dinv")
    for r in range(i["nr"]):
        Dinv[r * b:(r + 1) * b, r * b:(r + 1) * b] = Dv[r]
    return A, Dinv, i["lam"]


def _cheb_error(Z, sigma, k):
    """T_k(Z) / T_k(sigma) by the three-term recurrence T_{j+1} = 2 z T_j - T_{j-1}."""
    I = np.eye(Z.shape[0])
    Tm, T = I, Z
    tm, t = 1.0, sigma
    for _ in range(k - 1):
        Tm, T = T, 2 * Z @ T - Tm
        tm, t = t, 2 * sigma * t - tm
    return T / t


@pytest.mark.parametrize("degree", [2, 5])
def test_chebyshev_smoother_error_is_the_chebyshev_polynomial(degree):
    rp, ci, val, _ = _laplacian_box(4, 4, 3)
    n = rp.size - 1
    h = oracle.Amg(rp, ci, val, np.ones((n, 1)), oracle.amg_opts(coarse_max=10, theta=0.05, cheb_degree=degree))
    A, Dinv, lam = _dense_level(h, 0)
    lmax, lmin = lam, lam / 30
    theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
    Y = Dinv @ A
    I = np.eye(n)
    Z = (theta * I - Y) / delta
    E = _cheb_error(Z, theta / delta, degree)
    rng = np.random.default_rng(2)
    b = rng.normal(size=n)
    x = h.smooth(0, b)
    xs = np.linalg.solve(A, b)
    assert np.allclose(x, (I - E) @ xs, atol=1e-12 * np.abs(xs).max())
    # from a nonzero start the error is propagated by the same polynomial
    x0 = rng.normal(size=n)
    x1 = h.smooth(0, b, x0)
    assert np.allclose(xs - x1, E @ (xs - x0), atol=1e-11 * np.abs(xs - x0).max())


def test_jacobi_smoother_two_sweeps():
    rp, ci, val, _ = _laplacian_box(4, 3, 3)
    n = rp.size - 1
    h = oracle.Amg(rp, ci, val, np.ones((n, 1)), oracle.amg_opts(coarse_max=10, smoother=0, theta=0.05))
    A, Dinv, lam = _dense_level(h, 0)
    w = 4 / (3 * lam)
    E = np.eye(n) - w * Dinv @ A
    b = np.random.default_rng(3).normal(size=n)
    xs = np.linalg.solve(A, b)
    assert np.allclose(h.smooth(0, b), xs - E @ E @ xs, atol=1e-12 * np.abs(xs).max())


@pytest.mark.parametrize("smoother", [0, 1])
def test_vcycle_is_symmetric_and_matches_two_grid_formula(scr_small, smoother, small_fsi):
    o = oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz,
                   oracle.amg_opts(coarse_max=200, smoother=smoother, max_levels=2))
    h = o.amgA
    assert h.nlevels == 2
    A, Dinv, lam = _dense_level(h, 0)
    n = A.shape[0]
    M = np.column_stack([h.vcycle(e) for e in np.eye(n)])
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
    # two-grid: x = S_post(b, x_pre + P Ac^-1 R (b - A x_pre)) with x_pre = S_pre(b, 0)
    P = bsr_to_dense(h.get(0, "P.rp"), h.get(0, "P.ci"), h.get(0, "P.v"), h.info(0)["nagg"])
    Ac = bsr_to_dense(h.get(1, "A.rp"), h.get(1, "A.ci"), h.get(1, "A.v"), h.info(1)["nr"])
    I = np.eye(n)
    if smoother == 1:
        lmax, lmin = lam, lam / 30
        th, de = (lmax + lmin) / 2, (lmax - lmin) / 2
        Z = (th * I - Dinv @ A) / de
        E = _cheb_error(Z, th / de, oracle.amg_opts().cheb_degree)
    else:
        Ej = I - 4 / (3 * lam) * Dinv @ A
        E = Ej @ Ej
    Ainv = np.linalg.inv(A)
    Ecg = I - P @ np.linalg.solve(Ac, P.T @ A)
    Etg = E @ Ecg @ E                                   # error propagation of the two-grid cycle
    assert np.abs((I - M @ A) - Etg).max() <= 1e-9 * max(1, np.abs(Etg).max())


# ----------------------------------------------------------------------------- Krylov
def test_gmres_minimal_residual_property():
    rng = np.random.default_rng(5)
    rp, ci, val, _ = _laplacian_box(3, 3, 3)
    n = rp.size - 1
    val = val + 0.3 * rng.normal(size=val.size) * (np.repeat(np.arange(n), np.diff(rp)) != ci)   # nonsymmetric
    A = bsr_to_dense(rp, ci, val, n)
    b = rng.normal(size=n)
    for k in (1, 3, 7):
        x, rc, its, rel = oracle.gmres(rp, ci, val, b, tol=1e-30, maxit=k, restart=50)
        assert its == k
        Kb = np.column_stack([np.linalg.matrix_power(A, j) @ b for j in range(k)])
        y = np.linalg.lstsq(A @ Kb, b, rcond=None)[0]
        best = np.linalg.norm(b - A @ Kb @ y)
        assert np.linalg.norm(b - A @ x) == pytest.approx(best, rel=1e-7)
    x, rc, its, rel = oracle.gmres(rp, ci, val, b, tol=1e-12, maxit=500, restart=10)
    assert rc == 0 and np.allclose(x, np.linalg.solve(A, b), atol=1e-9)


def test_cg_iteration_bound_from_closed_form_spectrum():
    nx = ny = nz = 8
    rp, ci, val, s = _laplacian_box(nx, ny, nz)
    b = synth.rhs(1, rp.size - 1, s.Lmask)
    n = [nx - 1, ny - 1, nz - 1]
    lmin = 6 * sum(4 * np.sin(np.pi / (2 * (m + 1))) ** 2 for m in n)
    lmax = 6 * sum(4 * np.sin(m * np.pi / (2 * (m + 1))) ** 2 for m in n)
    kappa = max(lmax, 1.0) / min(lmin, 1.0)            # Dirichlet identity rows have eigenvalue 1
    eps = 1e-8
    bound = int(np.ceil(0.5 * np.sqrt(kappa) * np.log(2 / eps))) + 1
    x, rc, its, rel = oracle.cg(rp, ci, val, b, tol=eps, maxit=1000)
    assert rc == 0 and its <= bound
    A = bsr_to_dense(rp, ci, val)
    assert np.linalg.norm(b - A @ x) <= eps * np.linalg.norm(b) * (1 + 1e-6)
    # flexible CG equals PCG for a fixed preconditioner
    h = oracle.Amg(rp, ci, val, np.ones((rp.size - 1, 1)), oracle.amg_opts(coarse_max=40, theta=0.05))
    x1, _, i1, _ = oracle.cg(rp, ci, val, b, amg=h, tol=1e-10)
    x2, _, i2, _ = oracle.cg(rp, ci, val, b, amg=h, tol=1e-10, flexible=True)
    assert i1 == i2 and np.allclose(x1, x2, atol=1e-9 * np.abs(x1).max())
    assert i1 < its


# ----------------------------------------------------------------------------- S^, Algorithm 2, Algorithm 1
def _dense_blocks(s):
    nb = s.n_b
    Kd = bsr_to_dense(s.rp, s.ci, s.val)
    perm = split_perm(nb)
    Ks = Kd[np.ix_(perm, perm)]
    return Ks[:3 * nb, :3 * nb], Ks[:3 * nb, 3 * nb:], Ks[3 * nb:, :3 * nb], Ks[3 * nb:, 3 * nb:], Kd, perm


def test_schur_approximation_brute_force(tiny):
    o = oracle.Scr(tiny.rp, tiny.ci, tiny.val, tiny.xyz)
    A, G, D, Cb, _, _ = _dense_blocks(tiny)
    Sd = Cb - D @ np.diag(1 / np.diag(A)) @ G
    rp, ci, v = o.matrix("Shat")
    S = bsr_to_dense(rp, ci, v, tiny.n_b)
    assert np.abs(S - Sd).max() <= 1e-13 * np.abs(Sd).max()
    assert np.allclose(S, S.T, atol=1e-14 * np.abs(S).max()) and np.linalg.eigvalsh(S).min() > 0
    for name, M in (("A", A), ("G", G), ("D", D), ("C", Cb)):
        rp, ci, v = o.matrix(name)
        assert np.array_equal(bsr_to_dense(rp, ci, v, tiny.n_b), M)


def test_algorithm2_matrix_free_schur(small_fsi):
    o = oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz)
    A, G, D, Cb, _, _ = _dense_blocks(small_fsi)
    xp = np.random.default_rng(6).normal(size=small_fsi.n_b)
    exact = Cb @ xp - D @ np.linalg.solve(A, G @ xp)
    y = o.apply("S", xp, oracle.solve_opts(tol_I=1e-14))
    assert np.linalg.norm(y - exact) <= 1e-10 * np.linalg.norm(exact)
    # loose inner tolerance gives a perturbed action, not the exact one
    y3 = o.apply("S", xp, oracle.solve_opts(tol_I=1e-2))
    assert np.linalg.norm(y3 - exact) > 1e-8 * np.linalg.norm(exact)


def test_algorithm1_with_exact_inner_solves_is_the_inverse(small_fsi):
    # Block LDU (Sec. 5.2.1): with exact A and S solves, P_SCR^-1 = A^-1 (the 2x2 system's inverse)
    o = oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz)
    A, G, D, Cb, Kd, perm = _dense_blocks(small_fsi)
    Ks = np.block([[A, G], [D, Cb]])
    r = np.random.default_rng(8).normal(size=4 * small_fsi.n_b)
    tight = oracle.solve_opts(tol_A=1e-14, tol_S=1e-14, tol_I=1e-14, max_it_S=400, max_it_A=400, max_it_I=400)
    y = o.apply("SCR", r, tight)
    exact = np.linalg.solve(Ks, r)
    assert np.linalg.norm(y - exact) <= 1e-9 * np.linalg.norm(exact)
    b = synth.rhs(2, 4 * small_fsi.n_b, small_fsi.mask)
    tight.tol = 1e-10
    x, rc, st = o.solve(b, tight)
    assert rc == 0 and st["outer_it"] == 1


# ----------------------------------------------------------------------------- SIMPLE / SIMPLEC (Sec. 5.2.1)
def test_simple_with_exact_solves_is_the_inverse_of_its_product_form(small_fsi):
    # P_SIMPLE = [I 0; D A^-1 I] [A 0; 0 S^] [I d^-1 G; 0 I], d = diag(A); its product closed form
    # is [A  A d^-1 G; D  C] (S^ = C - D d^-1 G), so it differs from the 2x2 system only in the
    # upper-right block
    o = oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz)
    A, G, D, Cb, _, _ = _dense_blocks(small_fsi)
    n3, nb = A.shape[0], Cb.shape[0]
    dinv = np.diag(1.0 / np.diag(A))
    Sh = Cb - D @ dinv @ G
    I3, Ip = np.eye(n3), np.eye(nb)
    P = (np.block([[I3, np.zeros((n3, nb))], [D @ np.linalg.inv(A), Ip]])
         @ np.block([[A, np.zeros((n3, nb))], [np.zeros((nb, n3)), Sh]])
         @ np.block([[I3, dinv @ G], [np.zeros((nb, n3)), Ip]]))
    closed = np.block([[A, A @ dinv @ G], [D, Cb]])
    assert np.abs(P - closed).max() <= 1e-9 * np.abs(closed).max()
    r = np.random.default_rng(9).normal(size=n3 + nb)
    tight = oracle.solve_opts(tol_A=1e-14, tol_S=1e-14, max_it_S=400, max_it_A=400)
    y = o.apply("SIMPLE", r, tight)
    exact = np.linalg.solve(closed, r)
    assert np.linalg.norm(y - exact) <= 1e-9 * np.linalg.norm(exact)


def test_simplec_lumped_diagonal_and_schur(tiny):
    # SIMPLEC: d = sums of the absolute values of the rows of A, used in S^ and in the update
    o = oracle.Scr(tiny.rp, tiny.ci, tiny.val, tiny.xyz, oracle.amg_opts(schur_diag=1))
    A, G, D, Cb, _, _ = _dense_blocks(tiny)
    d = np.abs(A).sum(axis=1)
    assert np.allclose(o.apply("d", np.zeros(A.shape[0])), d, rtol=1e-14, atol=0)
    rp, ci, v = o.matrix("Shat")
    S = bsr_to_dense(rp, ci, v, tiny.n_b)
    Sd = Cb - D @ np.diag(1.0 / d) @ G
    assert np.abs(S - Sd).max() <= 1e-13 * np.abs(Sd).max()
    o0 = oracle.Scr(tiny.rp, tiny.ci, tiny.val, tiny.xyz)
    assert np.array_equal(o0.apply("d", np.zeros(A.shape[0])), np.diag(A))


def test_simple_is_exact_when_A_is_diagonal(small_fsi):
    # with A = diag(A) the closed form [A  A d^-1 G; D  C] is the 2x2 system itself: FGMRES with
    # exact block solves converges in one iteration
    s = small_fsi
    val = s.val.copy()
    for r in range(s.n_b):
        for q in range(s.rp[r], s.rp[r + 1]):
            blk = val[q, :3, :3]
            keep = np.diag(np.diag(blk)) if s.ci[q] == r else np.zeros((3, 3))
            val[q, :3, :3] = keep
    o = oracle.Scr(s.rp, s.ci, val, s.xyz)
    b = synth.rhs(4, 4 * s.n_b, s.mask)
    opts = oracle.solve_opts(tol=1e-10, tol_A=1e-14, tol_S=1e-14, max_it_S=400, precond=1)
    x, rc, st = o.solve(b, opts)
    xl = oracle.dense_solve(bsr_to_dense(s.rp, s.ci, val), b)
    assert rc == 0 and st["outer_it"] == 1
    assert np.linalg.norm(x - xl) <= 1e-9 * np.linalg.norm(xl)


@pytest.mark.parametrize("schur_diag", [0, 1])
def test_simple_fgmres_matches_dense_lu(small_fsi, schur_diag):
    s = small_fsi
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(schur_diag=schur_diag))
    b = synth.rhs(3, 4 * s.n_b, s.mask)
    x, rc, st = o.solve(b, oracle.solve_opts(tol=1e-11, precond=1))
    xl = oracle.dense_solve(bsr_to_dense(s.rp, s.ci, s.val), b)
    assert rc == 0 and st["calls_I"] == 0 and st["calls_S"] == st["outer_it"]
    assert np.linalg.norm(x - xl) <= 1e-9 * np.linalg.norm(xl)


def test_full_solve_matches_dense_lu(tiny, small_fsi):
    for s in (tiny, small_fsi):
        o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
        Kd = bsr_to_dense(s.rp, s.ci, s.val)
        for seed in (0, 1):
            b = synth.rhs(seed, 4 * s.n_b, s.mask)
            # kappa(K) ~ 2e9 here: the attainable FP64 relative residual is ~1e-12, so 1e-11
            x, rc, st = o.solve(b, oracle.solve_opts(tol=1e-11))
            xl = oracle.dense_solve(Kd, b)
            assert rc == 0
            assert np.linalg.norm(x - xl) <= 1e-10 * np.linalg.norm(xl)
            assert np.linalg.norm(Kd @ xl - b) <= 1e-10 * np.linalg.norm(b)


def test_cfg0_solve_residual_and_manufactured_solution(cfg0):
    o = oracle.Scr(cfg0.rp, cfg0.ci, cfg0.val, cfg0.xyz)
    b = synth.rhs(0, 4 * cfg0.n_b, cfg0.mask)
    x, rc, st = o.solve(b)
    r = b - oracle.bsr_spmv(cfg0.rp, cfg0.ci, cfg0.val, x)
    assert rc == 0 and np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)
    assert st["rel_res_true"] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(b), rel=1e-6)
    xs = synth.rhs(11, 4 * cfg0.n_b, cfg0.mask)
    bs = oracle.bsr_spmv(cfg0.rp, cfg0.ci, cfg0.val, xs)
    x2, rc, st = o.solve(bs, oracle.solve_opts(tol=1e-12))
    assert rc == 0 and np.linalg.norm(x2 - xs) <= 1e-8 * np.linalg.norm(xs)


def test_not_converged_is_reported(cfg0):
    o = oracle.Scr(cfg0.rp, cfg0.ci, cfg0.val, cfg0.xyz)
    b = synth.rhs(0, 4 * cfg0.n_b, cfg0.mask)
    x, rc, st = o.solve(b, oracle.solve_opts(max_it=1))
    assert rc == 1 and st["outer_it"] == 1 and st["rel_res_true"] > 1e-8


# ----------------------------------------------------------------------------- mesh motion
def test_mesh_motion_cg_amg_matches_dense(small_fsi):
    s = small_fsi
    m = oracle.Mesh(s.Lrp, s.Lci, s.Lval, oracle.amg_opts(coarse_max=50))
    b = synth.rhs(3, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    x, rc, its, rel = m.solve(b, tol=1e-12)
    L = bsr_to_dense(s.Lrp, s.Lci, s.Lval)
    X = np.linalg.solve(L, b.reshape(-1, 3))
    assert rc == 0 and np.abs(x.reshape(-1, 3) - X).max() <= 1e-9 * np.abs(X).max()
    assert np.all(its > 0) and np.all(rel <= 1e-12)


# ----------------------------------------------------------------------------- numeric re-setup
_FIELDS = ("A.rp", "A.ci", "A.v", "agg", "strong", "dead", "P.rp", "P.ci", "P.v", "R.rp", "R.ci", "R.v", "Dinv", "B")


def _same_hierarchy(h1, h2):
    assert h1.nlevels == h2.nlevels
    for l in range(h1.nlevels):
        i1, i2 = h1.info(l), h2.info(l)
        assert i1 == i2, (l, i1, i2)
        fields = _FIELDS if l + 1 < h1.nlevels else ("A.rp", "A.ci", "A.v", "B")
        for f in fields:
            assert np.array_equal(h1.get(l, f), h2.get(l, f)), (l, f)


def _node_scaling(nb, seed):
    """powers of two per block row: a similarity S K S that changes every value but leaves
    every strength ratio exactly as it was"""
    return np.exp2(np.random.default_rng(seed).integers(-3, 4, nb)).astype(np.float64)


def test_update_with_the_same_values_is_identical(small_fsi):
    s = small_fsi
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(coarse_max=60))
    ref = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(coarse_max=60))
    o.update(s.val.copy())
    _same_hierarchy(o.amgA, ref.amgA)
    _same_hierarchy(o.amgS, ref.amgS)
    b = synth.rhs(2, 4 * s.n_b, s.mask)
    assert np.array_equal(o.solve(b)[0], ref.solve(b)[0])


@pytest.mark.parametrize("case", ["similarity_two_level", "uniform_scaling"])
def test_update_equals_a_fresh_setup_when_aggregates_coincide(small_fsi, case):
    # A numeric re-setup must reproduce a full setup exactly whenever the full setup would pick
    # the same aggregates, so that nothing value-dependent (d, S^, D^-1, lambda, P_tent, P, R,
    # RAP, dead dofs, coarse LU) is stale.  Two such changes:
    #  * K' = S K S with S a diagonal of powers of two per node: every value and every P changes,
    #    the level-0 strength ratios cannot (two-level hierarchies: only level 0 aggregates);
    #  * K' = 2 K: every level's strength ratios are unchanged (all levels).
    s = small_fsi
    rows = np.repeat(np.arange(s.n_b), np.diff(s.rp))
    if case == "similarity_two_level":
        sc = _node_scaling(s.n_b, 3)
        val2 = s.val * (sc[rows] * sc[s.ci])[:, None, None]
        ao = oracle.amg_opts(coarse_max=60, max_levels=2)
    else:
        val2 = 2.0 * s.val
        ao = oracle.amg_opts(coarse_max=60)
    fresh = oracle.Scr(s.rp, s.ci, val2, s.xyz, ao)
    upd = oracle.Scr(s.rp, s.ci, s.val, s.xyz, ao)
    upd.update(val2)
    _same_hierarchy(upd.amgA, fresh.amgA)
    _same_hierarchy(upd.amgS, fresh.amgS)
    for name in ("A", "G", "D", "C", "Shat"):
        for a, b_ in zip(upd.matrix(name), fresh.matrix(name)):
            assert np.array_equal(a, b_), name
    b = synth.rhs(5, 4 * s.n_b, s.mask)
    x1, rc1, st1 = upd.solve(b)
    x2, rc2, st2 = fresh.solve(b)
    assert rc1 == rc2 == 0 and np.array_equal(x1, x2) and st1 == st2


def test_update_keeps_aggregates_for_a_changed_time_step(small_fsi):
    # a different dt changes the mass term, and a fresh setup would aggregate differently; the
    # re-setup keeps the old aggregates and still solves the new system
    s = small_fsi
    p2 = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0, dt=2e-3)
    s2 = synth.generate(p2)
    assert np.array_equal(s.rp, s2.rp) and np.array_equal(s.ci, s2.ci)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz, oracle.amg_opts(coarse_max=60))
    agg0 = [o.amgA.get(l, "agg").copy() for l in range(o.amgA.nlevels - 1)]
    o.update(s2.val)
    for l, a in enumerate(agg0):
        assert np.array_equal(o.amgA.get(l, "agg"), a)
    b = synth.rhs(6, 4 * s.n_b, s2.mask)
    x, rc, st = o.solve(b, oracle.solve_opts(tol=1e-11))
    xl = oracle.dense_solve(bsr_to_dense(s2.rp, s2.ci, s2.val), b)
    assert rc == 0 and np.linalg.norm(x - xl) <= 1e-9 * np.linalg.norm(xl)


def test_mesh_update_equals_a_fresh_setup_when_aggregates_coincide(cfg0):
    s = cfg0
    sc = _node_scaling(s.n_phys, 4)
    rows = np.repeat(np.arange(s.n_phys), np.diff(s.Lrp))
    v2 = s.Lval * sc[rows] * sc[s.Lci]
    ao = oracle.amg_opts(max_levels=2, coarse_max=4000)
    fresh = oracle.Mesh(s.Lrp, s.Lci, v2, ao)
    upd = oracle.Mesh(s.Lrp, s.Lci, s.Lval, ao)
    upd.update(v2)
    _same_hierarchy(upd.amg, fresh.amg)


# ----------------------------------------------------------------------------- advection and outlets
@pytest.fixture(scope="module")
def flow_fsi():
    """small_fsi with the advective Poiseuille state (u_max = 30): a nonsymmetric velocity block."""
    kw = dict(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0)
    return synth.generate(synth.default_params(u_max=30.0, **kw))


def _outlet_columns(s, outlets):
    """the coupling vectors as dense interleaved 4n columns (velocity entries only)"""
    cols = []
    for blk, a in outlets:
        v = np.zeros((s.n_b, 4))
        v[blk, :3] = a
        cols.append(v.reshape(-1))
    return np.array(cols).T


def _two_outlets(s):
    blk, a = s.outlets[0]
    h = len(blk) // 2
    return [(blk[:h], a[:h]), (blk[h:], a[h:])], np.array([1.0e3, 4.0e3])


def test_advective_system_solve_matches_dense_lu(flow_fsi):
    s = flow_fsi
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    Kd = bsr_to_dense(s.rp, s.ci, s.val)
    b = synth.rhs(3, 4 * s.n_b, s.mask)
    x, rc, st = o.solve(b, oracle.solve_opts(tol=1e-11))
    xl = oracle.dense_solve(Kd, b)
    assert rc == 0 and np.linalg.norm(x - xl) <= 1e-10 * np.linalg.norm(xl)


def test_outlet_coupling_solve_is_the_woodbury_update_of_the_plain_solve(flow_fsi):
    # (K + U M U^T)^-1 b = y - Z (M^-1 + U^T Z)^-1 U^T y with y = K^-1 b, Z = K^-1 U: the plain
    # system's dense LU only, so nothing of the oracle's operator enters the reference
    s = flow_fsi
    outlets, m = _two_outlets(s)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    o.set_outlets(outlets, m)
    Kd = bsr_to_dense(s.rp, s.ci, s.val)
    U = _outlet_columns(s, outlets)
    b = synth.rhs(3, 4 * s.n_b, s.mask)
    y = oracle.dense_solve(Kd, b)
    Z = np.column_stack([oracle.dense_solve(Kd, U[:, k]) for k in range(U.shape[1])])
    xw = y - Z @ np.linalg.solve(np.diag(1.0 / m) + U.T @ Z, U.T @ y)
    x, rc, st = o.solve(b, oracle.solve_opts(tol=1e-11))
    assert rc == 0 and np.linalg.norm(x - xw) <= 1e-9 * np.linalg.norm(xw)
    assert np.linalg.norm(y - xw) > 1e-5 * np.linalg.norm(xw)         # the coupling matters here
    # swapping the two resistances is a different system
    o.set_outlets(outlets, m[::-1])
    x2, _, _ = o.solve(b, oracle.solve_opts(tol=1e-11))
    assert np.linalg.norm(x2 - xw) > 1e-6 * np.linalg.norm(xw)
    # removing the coupling restores the plain solve
    o.set_outlets([], [])
    x0, rc0, _ = o.solve(b, oracle.solve_opts(tol=1e-11))
    assert rc0 == 0 and np.linalg.norm(x0 - y) <= 1e-9 * np.linalg.norm(y)


def test_algorithm2_with_outlets_uses_the_coupled_velocity_block(flow_fsi):
    # S x = C x - D (A + sum_k m_k a_k a_k^T)^-1 G x with exact inner solves
    s = flow_fsi
    outlets, m = _two_outlets(s)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    o.set_outlets(outlets, m)
    A, G, D, Cb, _, perm = _dense_blocks(s)
    Uv = _outlet_columns(s, outlets)[perm][:3 * s.n_b]
    Af = A + Uv @ np.diag(m) @ Uv.T
    xp = np.random.default_rng(9).normal(size=s.n_b)
    exact = Cb @ xp - D @ np.linalg.solve(Af, G @ xp)
    y = o.apply("S", xp, oracle.solve_opts(tol_I=1e-14, max_it_I=400))
    assert np.linalg.norm(y - exact) <= 1e-10 * np.linalg.norm(exact)
    plain = Cb @ xp - D @ np.linalg.solve(A, G @ xp)
    assert np.linalg.norm(plain - exact) > 1e-6 * np.linalg.norm(exact)
    # the A and K operators
    xv = np.random.default_rng(10).normal(size=3 * s.n_b)
    assert np.allclose(o.apply("A", xv), Af @ xv, rtol=0, atol=1e-12 * np.abs(Af @ xv).max())


# ----------------------------------------------------------------------------- near-null space of AMG(A)
def _p1_gradients(x4):
    """Gradients of the four P1 shape functions of a tetrahedron (rows), from J^-1."""
    J = (x4[1:] - x4[0]).T                       # columns x_a - x_0, a = 1..3
    G = np.linalg.inv(J)                         # row a - 1 of J^-1 is grad N_a, a = 1..3
    return np.vstack([-G.sum(0), G])


def _rigid_mode_errors(s, B):
    """For each column of the velocity near-null space B ((3 n_b) x 6), the largest symmetric
    gradient of its P1 interpolant over the mesh's elements, relative to the largest gradient;
    and the constant skew part (the rotation vector) of each column's gradient."""
    sym = np.zeros(B.shape[1]); skew = np.zeros((B.shape[1], 3)); gmax = np.zeros(B.shape[1])
    for e in range(s.n_tets):
        rows = s.tv[e]
        dN = _p1_gradients(s.xyz[rows])
        for c in range(B.shape[1]):
            u = B[:, c].reshape(-1, 3)[rows]     # nodal velocities of the element (4 x 3)
            grad = u.T @ dN                      # du_i/dx_j
            sym[c] = max(sym[c], np.abs(grad + grad.T).max() / 2)
            gmax[c] = max(gmax[c], np.abs(grad).max())
            w = (grad - grad.T) / 2
            skew[c] = (w[2, 1], w[0, 2], w[1, 0])
    return sym, gmax, skew


@pytest.mark.parametrize("which", ["small_fsi", "cfg0"])
def test_near_null_space_of_A_is_the_six_rigid_motions(which, request):
    # Sec. 5.2.1 preconditions A with AMG(A); its near-null space must be the rigid motions that
    # the deviatoric operator annihilates: three translations (zero gradient, value e_c) and
    # three rotations (zero symmetric gradient, constant skew gradient about z, x, y).
    s = request.getfixturevalue(which)
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    B = o.amgA.get(0, "B")
    assert B.shape == (3 * s.n_b, 6)
    sym, gmax, skew = _rigid_mode_errors(s, B)
    assert np.all(sym <= 1e-12 * np.maximum(gmax, 1.0)), sym
    for c in range(3):
        assert gmax[c] <= 1e-12
        assert np.array_equal(B[:, c].reshape(-1, 3), np.tile(np.eye(3)[c], (s.n_b, 1)))
    for c, axis in zip(range(3, 6), (2, 0, 1)):
        assert np.allclose(skew[c], np.eye(3)[axis], atol=1e-12)
    # the six columns are independent on the mesh
    assert np.linalg.matrix_rank(B) == 6


def test_near_null_space_check_catches_a_flipped_rotation_sign(small_fsi):
    # the check above is sensitive: one sign flipped in a rotation column breaks it
    s = small_fsi
    o = oracle.Scr(s.rp, s.ci, s.val, s.xyz)
    B = o.amgA.get(0, "B").copy()
    Bv = B.reshape(-1, 3, 6)
    Bv[:, 1, 3] = -Bv[:, 1, 3]                   # u = (-y, x, 0) becomes (-y, -x, 0)
    sym, gmax, _ = _rigid_mode_errors(s, Bv.reshape(-1, 6))
    assert sym[3] > 0.5 and np.all(sym[[0, 1, 2, 4, 5]] <= 1e-12 * np.maximum(gmax[[0, 1, 2, 4, 5]], 1.0))


def test_deviatoric_and_graddiv_operators_annihilate_the_near_null_space(small_fsi):
    # the generator's viscous/elastic (deviatoric) and grad-div terms alone, with natural
    # boundaries, have the oracle's six near-null vectors in their kernel on every velocity row
    # of a physical node (the rows of virtual interface nodes are identity rows)
    p = synth.default_params(mode=0, m_core=2, n_bl=1, n_wall=1, nz=8, R=1.0, L=2.0, terms=2 | 4, apply_bc=0)
    s = synth.generate(p, tets=True)
    assert s.n_b == small_fsi.n_b and np.array_equal(s.xyz, small_fsi.xyz)
    o = oracle.Scr(small_fsi.rp, small_fsi.ci, small_fsi.val, small_fsi.xyz)
    B = o.amgA.get(0, "B")
    A = s.val[:, :3, :3]
    AB = np.stack([oracle.bsr_spmv(s.rp, s.ci, A, B[:, c]) for c in range(6)], axis=1)
    phys = np.repeat(s.kind != 3, 3)
    scale = np.abs(A).max() * np.abs(B).max() * 15
    assert np.abs(AB[phys]).max() <= 1e-12 * scale
    # the full velocity block (mass included) does not annihilate them: the check has teeth
    Af = small_fsi.val[:, :3, :3]
    ABf = oracle.bsr_spmv(small_fsi.rp, small_fsi.ci, Af, B[:, 0])
    assert np.abs(ABf[phys]).max() > 1e-3 * scale


# ----------------------------------------------------------------------------- block strength
def _scaled_block(rng, b, f):
    """A random b x b block whose squared Frobenius norm is exactly f (to rounding)."""
    M = rng.normal(size=(b, b))
    return M * np.sqrt(f / (M * M).sum())


@pytest.mark.parametrize("b", [3, 6])
def test_block_strength_flips_at_the_frobenius_threshold(b):
    # strong iff f_ij^2 >= theta^4 f_ii f_jj with f the squared Frobenius norm of the block,
    # symmetrised by OR; blocks placed a relative 1e-6 above and below the threshold flip the
    # flag, whichever of (i, j) and (j, i) carries the coupling
    rng = np.random.default_rng(b)
    theta = 0.08
    fii, fjj = 3.7, 0.45
    thr = np.sqrt(theta ** 4 * fii * fjj)            # f_ij at the threshold
    rp = np.array([0, 2, 4], np.int32); ci = np.array([0, 1, 0, 1], np.int32)
    for side in (0, 1):                               # coupling in block (0,1) or in (1,0)
        for rel, expect in ((1 + 1e-6, 1), (1 - 1e-6, 0)):
            val = np.zeros((4, b, b))
            val[0] = _scaled_block(rng, b, fii)
            val[3] = _scaled_block(rng, b, fjj)
            val[1 + side] = _scaled_block(rng, b, rel * thr)
            val[2 - side] = _scaled_block(rng, b, 1e-3 * thr)   # the other direction is weak
            flags, iso = oracle.strength(rp, ci, val, theta)
            assert flags.tolist() == [0, expect, expect, 0], (side, rel, flags)
            assert iso.tolist() == [1 - expect, 1 - expect]
    # a norm other than the squared Frobenius norm would move the flip point: the max-abs entry
    # of a block scaled to the Frobenius threshold is well below it
    val = np.zeros((4, b, b))
    val[0] = _scaled_block(rng, b, fii); val[3] = _scaled_block(rng, b, fjj)
    val[1] = _scaled_block(rng, b, 1.001 * thr); val[2] = val[1].T
    assert (val[1] ** 2).max() < 0.9 * thr
    flags, _ = oracle.strength(rp, ci, val, theta)
    assert flags.tolist() == [0, 1, 1, 0]
