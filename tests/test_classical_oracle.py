"""Pins of the oracle's classical AMG (oracle.c, amg_type = 1: the preconditioner settings of the
paper's table in Sec. 5.2), against results fixed by the definitions and textbook cases:

* strength: the threshold's boundary (an entry at exactly theta times the row's largest negative
  coupling is strong, just below it is not), positive couplings, rows with a negative diagonal and
  the function (unknown) filter;
* HMIS: on one domain it is the Ruge-Stueben first pass, which gives every other point of the 1-D
  Laplacian and the red-black split of the 5-point Laplacian; on any domains every F point that
  influences some point depends on a C point; with one-row domains it is plain PMIS; the
  splitmix64 uniforms lie in [0, 1);
* extended+i: linear interpolation on a graded 1-D grid, for F points next to C points and for
  two F points in a row (the distance-two case, weights 2/3 and 1/3); rows of interpolation sum to
  one where the matrix's rows sum to zero (also after truncation); truncation and the five-entry
  cap on a star with known weights;
* aggressive coarsening: the second-stage graph equals the brute-force paths of length one or two
  among the C points (boolean matrix products); on the 1-D Laplacian two stages keep every fourth
  point and the two-stage interpolation is linear between them;
* hybrid Gauss-Seidel: one domain is Gauss-Seidel (triangular solves), one-row domains are Jacobi,
  general domains are block triangular solves with the previous iterate outside the block;
* the hierarchy: A_{l+1} = P^T A_l P in dense arithmetic, C rows of P the identity, the symmetry
  of the V-cycle (forward then backward sweeps) as an operator, and CG with it on the mesh
  Laplacian.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
import synth


def _csr(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def _lap1d(n, h=None):
    """1-D Laplacian (Dirichlet ends) on nodes with spacings h (n + 1 values): a_{i,i+-1} = -1/h."""
    h = np.ones(n + 1) if h is None else np.asarray(h)
    lo, hi = 1.0 / h[:-1], 1.0 / h[1:]
    return _csr(sp.diags([-lo[1:], lo + hi, -hi[:-1]], [-1, 0, 1], shape=(n, n)))


def _lap2d(n, eps=1.0):
    I = sp.eye(n)
    T = sp.diags([-1.0, 2.0, -1.0], [-1, 0, 1], shape=(n, n))
    return _csr(sp.kron(I, T) + eps * sp.kron(T, I))


def _strength(A, func=None, theta=0.5):
    func = np.zeros(A.shape[0], np.uint8) if func is None else func
    return oracle.cl_strength(A.indptr, A.indices, A.data, func, theta)


def _strong_dense(A, S):
    M = sp.csr_matrix((S.astype(float), A.indices, A.indptr), shape=A.shape)
    return M.toarray() > 0


# ------------------------------------------------------------------------------ strength
def test_strength_threshold_boundary_and_signs():
    for eps, strong_y in ((0.5, True), (0.5 * (1 - 1e-12), False), (0.3, False), (1.0, True)):
        A = _lap2d(4, eps)
        D = _strong_dense(A, _strength(A))
        # interior point 5 = (1, 1): x neighbours 4, 6 (coefficient -1), y neighbours 1, 9 (-eps)
        assert D[5, 4] and D[5, 6]
        assert D[5, 1] == strong_y and D[5, 9] == strong_y, eps
    # positive couplings are never strong; a negative diagonal flips the sign convention
    A = _csr(np.array([[4.0, -2.0, 1.0, -1.0], [-2.0, 4.0, 0.0, 0.0], [1.0, 0.0, 4.0, -3.0], [-1.0, 0.0, -3.0, 4.0]]))
    D = _strong_dense(A, _strength(A))
    assert D[0].tolist() == [False, True, False, True] and D[2].tolist() == [False, False, False, True]
    An = _csr(-A.toarray())
    assert np.array_equal(_strong_dense(An, _strength(An)), D)
    # no negative coupling: nothing strong
    A = _csr(np.array([[2.0, 1.0], [1.0, 2.0]]))
    assert not _strength(A).any()


def test_strength_only_within_a_function():
    A = _csr(np.array([[4.0, -10.0, -1.0, -0.6], [-10.0, 4.0, 0.0, 0.0], [-1.0, 0.0, 4.0, 0.0],
                       [-0.6, 0.0, 0.0, 4.0]]))
    func = np.array([0, 1, 0, 0], np.uint8)
    D = _strong_dense(A, _strength(A, func))
    # row 0: the -10 coupling is to another function and does not set the maximum
    assert D[0].tolist() == [False, False, True, True]
    assert not D[1].any()


# ------------------------------------------------------------------------------ HMIS
def test_one_domain_is_the_ruge_stueben_first_pass():
    A = _lap1d(11)
    cf, first = oracle.cl_hmis(A.indptr, A.indices, _strength(A), domain=1 << 20)
    assert np.array_equal(np.nonzero(cf > 0)[0], np.arange(1, 11, 2))
    assert np.array_equal(cf, first)
    A = _lap2d(8)
    cf, _ = oracle.cl_hmis(A.indptr, A.indices, _strength(A), domain=1 << 20)
    i, j = np.divmod(np.arange(64), 8)
    assert np.array_equal(cf > 0, (i + j) % 2 == 0)


def _check_split(A, S, cf):
    D = _strong_dense(A, S)
    np.fill_diagonal(D, False)
    influences = D.any(axis=0)                       # some point depends on i
    C = cf > 0
    for i in np.nonzero(~C & influences)[0]:
        assert (D[i] & C).any(), i


@pytest.mark.parametrize("domain", [1, 7, 64, 256, 1 << 20])
def test_every_influencing_f_point_depends_on_a_c_point(domain):
    s = synth.generate(synth.cfg0_params())
    L = _csr(sp.csr_matrix((s.Lval, s.Lci, s.Lrp)))
    for A in (L, _lap2d(12, 0.2)):
        S = _strength(A)
        cf, first = oracle.cl_hmis(A.indptr, A.indices, S, domain=domain, seed=3)
        _check_split(A, S, cf)
        if domain == 1:
            assert not (first > 0).any()            # one-row domains: nothing from the first pass
        assert 0 < (cf > 0).sum() < A.shape[0]


def test_pmis_uniforms():
    u = np.array([oracle.cl_uniform(5, 2, i) for i in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and len(np.unique(u)) == u.size
    assert oracle.cl_uniform(5, 2, 7) != oracle.cl_uniform(5, 3, 7) != oracle.cl_uniform(6, 2, 7)


# ------------------------------------------------------------------------------ ext+i
def _P(A, cf, func=None, trunc=0.3, pmax=5, theta=0.5):
    func = np.zeros(A.shape[0], np.uint8) if func is None else func
    S = _strength(A, func, theta)
    prp, pci, pv = oracle.cl_extpi(A.indptr, A.indices, A.data, func, S, np.asarray(cf, np.int8), trunc, pmax)
    return sp.csr_matrix((pv, pci, prp), shape=(A.shape[0], int((np.asarray(cf) > 0).sum()))).toarray()


def test_extpi_is_linear_interpolation_in_1d():
    # graded spacings (neighbouring couplings within a factor 2, so every coupling is strong)
    h = np.array([1.0, 0.8, 1.2, 1.0, 0.9, 1.3, 0.85, 1.05])
    x = np.concatenate([[0.0], np.cumsum(h)])[1:-1]        # interior nodes
    n = x.size
    A = _lap1d(n, h)
    # C F C F F C F: F next to C points, and a pair of F points (distance two)
    cf = np.array([1, -1, 1, -1, -1, 1, -1])
    P = _P(A, cf, trunc=0.0, pmax=0)
    Cx = x[cf > 0]
    for i in np.nonzero(cf < 0)[0]:
        # the piecewise-linear interpolant of the C values (f = x) and the zero Dirichlet ends
        lin = np.interp(x[i], np.concatenate([[0.0], Cx, [h.sum()]]), np.concatenate([[0.0], Cx, [0.0]]))
        assert P[i] @ Cx == pytest.approx(lin, rel=1e-14), i
    # uniform grid, C F F C: weights 2/3 and 1/3
    A = _lap1d(4)
    P = _P(A, [1, -1, -1, 1], trunc=0.0, pmax=0)
    assert np.allclose(P[1], [2 / 3, 1 / 3], rtol=0, atol=1e-15) and np.allclose(P[2], [1 / 3, 2 / 3], rtol=0, atol=1e-15)
    assert np.array_equal(P[[0, 3]], np.eye(2))


def test_extpi_rows_sum_to_one_for_zero_row_sums():
    p = synth.cfg0_params()
    p.apply_bc = 0
    s = synth.generate(p)
    L = _csr(sp.csr_matrix((s.Lval, s.Lci, s.Lrp)))
    assert np.abs(L @ np.ones(L.shape[0])).max() < 1e-12 * abs(L).max()
    S = _strength(L)
    cf, _ = oracle.cl_hmis(L.indptr, L.indices, S, domain=256)
    for trunc, pmax in ((0.0, 0), (0.3, 5), (0.5, 2)):
        P = _P(L, cf, trunc=trunc, pmax=pmax)
        rows = P.sum(axis=1)
        nonempty = (P != 0).any(axis=1)
        assert nonempty.mean() > 0.99
        assert np.abs(rows[nonempty] - 1.0).max() <= 1e-12, (trunc, pmax)
        nnz = (P != 0).sum(axis=1)
        if pmax:
            assert nnz.max() <= pmax
        # distance-two points are used (some F rows interpolate from C points that are not neighbours)
        if trunc == 0.0:
            Cidx = np.nonzero(cf > 0)[0]
            far = sum(1 for i in np.nonzero(cf < 0)[0] for j in np.nonzero(P[i])[0] if L[i, Cidx[j]] == 0)
            assert far > 0


def test_truncation_and_cap_on_a_star():
    # centre 0 (F) coupled to 7 C leaves with weights c_j, all strong (threshold 0.05); no F
    # neighbours: w_j = c_j / sum(c)
    c = np.array([5.0, 1.0, 3.0, 3.0, 0.5, 4.0, 2.0])
    n = c.size + 1
    A = np.zeros((n, n))
    A[0, 1:] = A[1:, 0] = -c
    A[0, 0] = c.sum()
    A[np.arange(1, n), np.arange(1, n)] = c + 1.0
    A = _csr(A)
    cf = np.array([-1] + [1] * c.size)
    w = c / c.sum()
    P = _P(A, cf, trunc=0.0, pmax=0, theta=0.05)
    assert np.allclose(P[0], w, rtol=1e-15, atol=0)
    # trunc 0.3: drop c < 1.5 (0.3 * 5), rescale to the row sum 1
    P = _P(A, cf, trunc=0.3, pmax=0, theta=0.05)
    keep = c >= 0.3 * c.max()
    assert np.allclose(P[0], np.where(keep, c / c[keep].sum(), 0.0), rtol=1e-15, atol=0)
    # cap 3: the three largest (5, 4, then the lower-column 3)
    P = _P(A, cf, trunc=0.3, pmax=3, theta=0.05)
    kept = np.zeros(c.size, bool); kept[[0, 2, 5]] = True
    assert np.allclose(P[0], np.where(kept, c / c[kept].sum(), 0.0), rtol=1e-15, atol=0)


# ------------------------------------------------------------------------------ aggressive coarsening
@pytest.mark.parametrize("which", ["lap2d", "mesh"])
def test_second_stage_graph_is_paths_of_length_two(which):
    if which == "lap2d":
        A = _lap2d(10, 0.3)
    else:
        s = synth.generate(synth.cfg0_params())
        A = _csr(sp.csr_matrix((s.Lval, s.Lci, s.Lrp)))
    S = _strength(A)
    cf, _ = oracle.cl_hmis(A.indptr, A.indices, S, domain=64)
    grp, gci, gS = oracle.cl_second_stage(A.indptr, A.indices, S, cf)
    D = sp.csr_matrix((S.astype(np.int64), A.indices, A.indptr), shape=A.shape)
    D.eliminate_zeros()
    C = np.nonzero(cf > 0)[0]
    reach = (D + D @ D).tocsr()[C][:, C].toarray() > 0     # paths of one or two strong dependencies
    E = reach.copy()
    np.fill_diagonal(E, False)
    n1 = C.size
    G = np.zeros((n1, n1), bool)
    F = np.zeros((n1, n1), bool)
    rows = np.repeat(np.arange(n1), np.diff(grp))
    G[rows, gci] = True
    F[rows, gci] = gS.astype(bool)
    assert np.array_equal(F, E)                      # the edges
    assert np.array_equal(G, E | E.T)                # the symmetric pattern
    assert all(np.all(np.diff(gci[grp[i]:grp[i + 1]]) > 0) for i in range(n1))


def test_aggressive_1d_keeps_every_fourth_point_and_interpolates_linearly():
    n = 31
    A = _lap1d(n)
    B = np.ones((n, 1))
    h = oracle.Amg(A.indptr, A.indices, A.data, B,
                   oracle.amg_opts(amg_type=1, agg_levels=1, coarse_max=4, hmis_domain=1 << 20, trunc=0.0, pmax=0))
    agg = h.get(0, "agg")
    C = np.nonzero(agg >= 0)[0]
    assert np.array_equal(C, np.arange(3, n, 4))
    i = h.info(0)
    P = sp.csr_matrix((h.get(0, "P.v").ravel(), h.get(0, "P.ci"), h.get(0, "P.rp")), shape=(n, i["nagg"])).toarray()
    x = np.arange(1, n + 1, dtype=float)           # node positions; zero Dirichlet values at 0 and n + 1
    lin = np.interp(x, np.concatenate([[0.0], x[C], [n + 1.0]]), np.concatenate([[0.0], x[C], [0.0]]))
    assert np.allclose(P @ x[C], lin, rtol=0, atol=1e-13)
    # the default truncation keeps the same rows here (weights 3/4 and 1/4 pass 0.3 of the largest)
    h2 = oracle.Amg(A.indptr, A.indices, A.data, B,
                    oracle.amg_opts(amg_type=1, agg_levels=1, coarse_max=4, hmis_domain=1 << 20))
    P2 = sp.csr_matrix((h2.get(0, "P.v").ravel(), h2.get(0, "P.ci"), h2.get(0, "P.rp")), shape=(n, i["nagg"])).toarray()
    assert np.allclose(P2, P, rtol=0, atol=1e-14)


def test_aggressive_levels_coarsen_faster_and_keep_galerkin():
    s = synth.generate(synth.cfg0_params())
    h0 = oracle.Mesh(s.Lrp, s.Lci, s.Lval, oracle.amg_opts(amg_type=1, agg_levels=0, coarse_max=64)).amg
    m2 = oracle.Mesh(s.Lrp, s.Lci, s.Lval, oracle.amg_opts(amg_type=1, agg_levels=2, coarse_max=64))
    h2 = m2.amg
    r0 = [h0.info(l)["nr"] for l in range(h0.nlevels)]
    r2 = [h2.info(l)["nr"] for l in range(h2.nlevels)]
    assert r2[1] < r0[1] / 2 and r2[2] < r0[2]
    op0 = sum(h0.info(l)["nnzA"] for l in range(h0.nlevels))
    op2 = sum(h2.info(l)["nnzA"] for l in range(h2.nlevels))
    assert op2 < op0                                   # lower operator complexity
    for l in range(2):
        i = h2.info(l)
        A = sp.csr_matrix((h2.get(l, "A.v").ravel(), h2.get(l, "A.ci"), h2.get(l, "A.rp")), shape=(i["nr"],) * 2)
        P = sp.csr_matrix((h2.get(l, "P.v").ravel(), h2.get(l, "P.ci"), h2.get(l, "P.rp")), shape=(i["nr"], i["nagg"]))
        j = h2.info(l + 1)
        Ac = sp.csr_matrix((h2.get(l + 1, "A.v").ravel(), h2.get(l + 1, "A.ci"), h2.get(l + 1, "A.rp")),
                           shape=(j["nr"],) * 2).toarray()
        ref = P.toarray().T @ A.toarray() @ P.toarray()
        assert np.abs(Ac - ref).max() <= 1e-12 * np.abs(ref).max()
        assert (np.diff(P.indptr) <= 5).all()
    b = synth.rhs(2, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    x, rc, its, rel = m2.solve(b, tol=1e-10)
    assert rc == 0 and its.max() <= 40


# ------------------------------------------------------------------------------ hybrid GS
def test_hybrid_gauss_seidel_special_cases():
    rng = np.random.default_rng(0)
    A = _lap2d(9) + sp.diags(rng.uniform(0.1, 1.0, 81))
    A = _csr(A)
    Ad = A.toarray()
    b = rng.standard_normal(81)
    x0 = rng.standard_normal(81)
    Lo, Up, D = np.tril(Ad, -1), np.triu(Ad, 1), np.diag(np.diag(Ad))
    # one domain: Gauss-Seidel forward / backward
    xf = oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=1 << 20)
    assert np.allclose(xf, sla.solve_triangular(D + Lo, b - Up @ x0, lower=True), rtol=1e-13, atol=1e-13)
    xb = oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=1 << 20, backward=True)
    assert np.allclose(xb, sla.solve_triangular(D + Up, b - Lo @ x0, lower=False), rtol=1e-13, atol=1e-13)
    # one-row domains: Jacobi
    xj = oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=1)
    assert np.allclose(xj, (b - (Ad - D) @ x0) / np.diag(Ad), rtol=1e-14, atol=1e-14)
    # domains of 16: triangular solve on each diagonal block, previous iterate elsewhere
    for backward in (False, True):
        x = oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=16, backward=backward)
        ref = np.empty(81)
        for lo in range(0, 81, 16):
            hi = min(81, lo + 16)
            blk = Ad[lo:hi, lo:hi]
            T = np.tril(blk) if not backward else np.triu(blk)
            rest = b[lo:hi] - Ad[lo:hi] @ x0 + T @ x0[lo:hi]
            ref[lo:hi] = sla.solve_triangular(T, rest, lower=not backward)
        assert np.allclose(x, ref, rtol=1e-13, atol=1e-13)
    # zero previous iterate
    assert np.allclose(oracle.cl_gs(A.indptr, A.indices, A.data, b, None, domain=1 << 20),
                       sla.solve_triangular(D + Lo, b, lower=True), rtol=1e-13, atol=1e-13)


def _ell(Ad, dom):
    """The l1 term of every row by its definition: s_i times the sum of |a_ij| over the columns of
    other domains."""
    n = Ad.shape[0]
    e = np.array([sum(abs(Ad[i, j]) for j in range(n) if j // dom != i // dom) for i in range(n)])
    return np.sign(np.diag(Ad)) * e


def test_l1_hybrid_gauss_seidel_special_cases():
    rng = np.random.default_rng(1)
    A = _csr(_lap2d(9) + sp.diags(rng.uniform(0.1, 1.0, 81)))
    Ad = A.toarray()
    b = rng.standard_normal(81)
    x0 = rng.standard_normal(81)
    # one domain: no coupling leaves it, the l1 sweep is the plain one
    for backward in (False, True):
        assert np.array_equal(oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=1 << 20, backward=backward, l1=True),
                              oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=1 << 20, backward=backward))
    # one-row domains: l1 Jacobi, x0 + (b - A x0) / (a_ii + sum_{j != i} |a_ij|)
    xj = oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=1, l1=True)
    l1d = np.diag(Ad) + (np.abs(Ad).sum(1) - np.abs(np.diag(Ad)))
    assert np.allclose(xj, x0 + (b - Ad @ x0) / l1d, rtol=1e-13, atol=1e-13)
    # domains of 16: x0 + M^-1 (b - A x0), M = the in-domain triangle of A plus diag(ell)
    ell = _ell(Ad, 16)
    for backward in (False, True):
        x = oracle.cl_gs(A.indptr, A.indices, A.data, b, x0, domain=16, backward=backward, l1=True)
        M = np.zeros_like(Ad)
        for lo in range(0, 81, 16):
            hi = min(81, lo + 16)
            blk = Ad[lo:hi, lo:hi]
            M[lo:hi, lo:hi] = np.triu(blk) if backward else np.tril(blk)
        M += np.diag(ell)
        ref = x0 + sla.solve_triangular(M, b - Ad @ x0, lower=not backward)
        assert np.allclose(x, ref, rtol=1e-12, atol=1e-12)
    # zero previous iterate: the l1 terms only enter through the diagonal
    M = np.tril(Ad) * (np.arange(81)[:, None] // 16 == np.arange(81)[None, :] // 16) + np.diag(ell)
    assert np.allclose(oracle.cl_gs(A.indptr, A.indices, A.data, b, None, domain=16, l1=True),
                       sla.solve_triangular(M, b, lower=True), rtol=1e-12, atol=1e-12)


def test_l1_sweep_converges_where_the_plain_one_diverges():
    # symmetric positive definite with positive couplings and D^-1 A reaching about 7: the plain
    # hybrid sweep (Jacobi between domains) amplifies the energy norm of the error, the l1 sweep
    # lowers it at every sweep (Baker, Falgout, Kolev and Yang)
    rng = np.random.default_rng(3)
    n = 512
    rows = np.repeat(np.arange(n), 6)
    S = sp.csr_matrix((rng.uniform(0.5, 1.0, n * 6), (rows, rng.integers(0, n, n * 6))), shape=(n, n))
    A = _csr(S @ S.T + 0.01 * sp.identity(n))
    x0 = rng.standard_normal(n)
    zero = np.zeros(n)
    for l1 in (False, True):
        x, en = x0.copy(), [x0 @ (A @ x0)]
        for k in range(12):
            x = oracle.cl_gs(A.indptr, A.indices, A.data, zero, x, domain=16, backward=bool(k % 2), l1=l1)
            en.append(x @ (A @ x))
        ratios = np.array(en[1:]) / np.array(en[:-1])
        if l1:
            assert ratios.max() < 1.0, ratios
        else:
            assert en[-1] > 1e3 * en[0], ratios


def test_hierarchy_uses_the_l1_diagonal():
    s = synth.generate(synth.cfg0_params())
    for l1 in (0, 1):
        m = oracle.Mesh(s.Lrp, s.Lci, s.Lval, oracle.amg_opts(amg_type=1, coarse_max=64, l1_gs=l1))
        h = m.amg
        for l in range(h.nlevels - 1):
            n = h.info(l)["nr"]
            A = sp.csr_matrix((h.get(l, "A.v").reshape(-1), h.get(l, "A.ci"), h.get(l, "A.rp")), shape=(n, n))
            if n <= 2000:
                Ad = A.toarray()
                d = np.diag(Ad) + (_ell(Ad, 64) if l1 else 0.0)
            else:
                # the dense definition is slow at the finest level: the same sums over the entries
                C = A.tocoo()
                off = (C.row // 64 != C.col // 64) & (C.row != C.col) if l1 else np.zeros(C.nnz, bool)
                e = np.bincount(C.row[off], np.abs(C.data[off]), minlength=n)
                d = A.diagonal() + np.sign(A.diagonal()) * e
            assert np.allclose(h.get(l, "Dinv").reshape(-1), 1.0 / d, rtol=1e-14, atol=0), (l1, l)


# ------------------------------------------------------------------------------ hierarchy
def test_hierarchy_galerkin_products_and_symmetric_cycle():
    s = synth.generate(synth.cfg0_params())
    o = oracle.amg_opts(amg_type=1, coarse_max=64)
    m = oracle.Mesh(s.Lrp, s.Lci, s.Lval, o)
    h = m.amg
    assert h.nlevels >= 3
    for l in range(h.nlevels - 1):
        i = h.info(l)
        A = sp.csr_matrix((h.get(l, "A.v").ravel(), h.get(l, "A.ci"), h.get(l, "A.rp")), shape=(i["nr"],) * 2)
        P = sp.csr_matrix((h.get(l, "P.v").ravel(), h.get(l, "P.ci"), h.get(l, "P.rp")), shape=(i["nr"], i["nagg"]))
        j = h.info(l + 1)
        Ac = sp.csr_matrix((h.get(l + 1, "A.v").ravel(), h.get(l + 1, "A.ci"), h.get(l + 1, "A.rp")),
                           shape=(j["nr"],) * 2)
        ref = P.toarray().T @ A.toarray() @ P.toarray()
        assert np.abs(Ac.toarray() - ref).max() <= 1e-12 * np.abs(ref).max()
        agg = h.get(l, "agg")
        Pd = P.toarray()
        for r in np.nonzero(agg >= 0)[0]:
            e = np.zeros(i["nagg"]); e[agg[r]] = 1.0
            assert np.array_equal(Pd[r], e)
        assert np.array_equal(np.sort(agg[agg >= 0]), np.arange(i["nagg"]))
    rng = np.random.default_rng(1)
    v, w = rng.standard_normal((2, s.n_phys))
    assert v @ h.vcycle(w) == pytest.approx(w @ h.vcycle(v), rel=1e-12)
    b = synth.rhs(2, 3 * s.n_phys, np.repeat(s.Lmask, 3))
    x, rc, its, rel = m.solve(b, tol=1e-10)
    Lm = sp.csr_matrix((s.Lval, s.Lci, s.Lrp))
    assert rc == 0 and its.max() <= 30
    assert np.linalg.norm(b.reshape(-1, 3) - Lm @ x.reshape(-1, 3)) <= 1e-9 * np.linalg.norm(b)


def test_classical_scr_solve_and_system_functions():
    s = synth.generate(synth.cfg0_params(), tets=True)
    o = oracle.amg_opts(amg_type=1)
    sc = oracle.Scr(s.rp, s.ci, s.val, s.xyz, o)
    func = sc.amgA.get(0, "func")
    assert np.array_equal(func, np.tile([0, 1, 2], s.n_b))
    # coarse points keep the function of their fine point
    agg = sc.amgA.get(0, "agg")
    f1 = sc.amgA.get(1, "func")
    assert np.array_equal(f1[agg[agg >= 0]], func[agg >= 0])
    # strength never couples two functions
    A0 = (sc.amgA.get(0, "A.rp"), sc.amgA.get(0, "A.ci"))
    S0 = sc.amgA.get(0, "strong")
    rows = np.repeat(np.arange(3 * s.n_b), np.diff(A0[0]))
    assert not (S0.astype(bool) & (func[rows] != func[A0[1]])).any()
    b = synth.rhs(4, 4 * s.n_b, s.mask)
    x, rc, st = sc.solve(b)
    assert rc == 0 and st["rel_res_true"] <= 1e-8
