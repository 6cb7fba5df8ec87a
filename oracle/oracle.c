/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the SCR+AMG linear-solve path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the GPU library (no headers, kernels,
 * helpers or constants); it is written from the paper's statements and from the published
 * methods it names, with no blocking, fusion or reordering beyond those definitions.
 *
 * What it computes (FP64 throughout):
 *   - dense LU with partial pivoting (reference solutions of tiny systems);
 *   - block split of the 2x2 system [A G; D C] (Sec. 5.2.1; the paper writes [A B; C D]);
 *   - the sparse Schur approximation S^ = C - D diag(A)^-1 G (Sec. 5.2.1, definition of S^);
 *   - smoothed-aggregation AMG (Vanek-Mandel-Brezina): strength graph, distance-2 maximal
 *     independent set by sequential greedy selection in descending seeded-key order,
 *     aggregation, Gram-Schmidt tentative prolongator on the near-null space, Jacobi-smoothed
 *     prolongator, Galerkin R*A*P, V-cycle with Chebyshev or damped block-Jacobi smoothing and
 *     a dense LU on the coarsest level;
 *   - right-preconditioned flexible GMRES(m) with modified Gram-Schmidt and Givens rotations
 *     (Saad 1993, which the paper uses at every level, Sec. 5.2.1);
 *   - the SCR preconditioner (Appendix B, Algorithm 1, step 2 read as r_p <- r_p - D y^_v) and
 *     the matrix-free Schur action (Appendix B, Algorithm 2);
 *   - preconditioned (and flexible) CG for the mesh-motion Laplacian (Sec. 5.2.2).
 * The parameters of SA-AMG are not in the paper (it uses BoomerAMG); they are inputs here.
 *
 * Threads (OpenMP) only split loops whose iterations are independent (rows of a product, entries
 * of a vector update, aggregates); every dot product sums fixed chunks of DOT_CHUNK entries in
 * order and then the chunk sums in order.  Every result is therefore the same for any thread
 * count, bit for bit.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* loops shorter than this run on one thread (thread start-up would dominate) */
#define PAR_MIN 4096
/* dot products: partial sums over fixed chunks of this many entries, then over the chunks */
#define DOT_CHUNK 4096

/* threads the parallel loops use (OMP_NUM_THREADS, else every core) */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ sparse block matrix */
typedef struct {
    int64_t nr, nc;
    int br, bc;
    int64_t nnzb;
    int32_t *rp, *ci;
    double* v;
} bsr;

static bsr* bsr_new(int64_t nr, int64_t nc, int br, int bc, int64_t nnzb) {
    bsr* M = (bsr*)calloc(1, sizeof(bsr));
    M->nr = nr; M->nc = nc; M->br = br; M->bc = bc; M->nnzb = nnzb;
    M->rp = (int32_t*)calloc(nr + 1, sizeof(int32_t));
    M->ci = (int32_t*)malloc(sizeof(int32_t) * (nnzb > 0 ? nnzb : 1));
    M->v = (double*)calloc((size_t)(nnzb > 0 ? nnzb : 1) * br * bc, sizeof(double));
    return M;
}
static void bsr_free(bsr* M) {
    if (!M) return;
    free(M->rp); free(M->ci); free(M->v); free(M);
}

/* y = M x */
static void bsr_mv(const bsr* M, const double* x, double* y) {
    int br = M->br, bc = M->bc;
#pragma omp parallel for schedule(static) if (M->nr > PAR_MIN)
    for (int64_t i = 0; i < M->nr; ++i) {
        double acc[8] = {0};
        for (int32_t q = M->rp[i]; q < M->rp[i + 1]; ++q) {
            const double* blk = M->v + (int64_t)q * br * bc;
            const double* xj = x + (int64_t)M->ci[q] * bc;
            for (int r = 0; r < br; ++r)
                for (int c = 0; c < bc; ++c) acc[r] += blk[r * bc + c] * xj[c];
        }
        for (int r = 0; r < br; ++r) y[i * br + r] = acc[r];
    }
}

static int32_t find_in_row(const bsr* M, int64_t i, int32_t c) {
    int32_t lo = M->rp[i], hi = M->rp[i + 1];
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (M->ci[mid] < c) lo = mid + 1; else hi = mid;
    }
    return (lo < M->rp[i + 1] && M->ci[lo] == c) ? lo : -1;
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* C = X * Y with the structural pattern (no numerical dropping), columns sorted.  Each row of C
 * is computed on its own (a row's terms are accumulated in the order of X's row, then of Y's
 * rows), so the rows are split over threads, each with its own column marks. */
static bsr* spgemm(const bsr* X, const bsr* Y) {
    int m = X->br, n = X->bc, p = Y->bc;
    int64_t nr = X->nr, nc = Y->nc;
    int32_t* rp = (int32_t*)calloc(nr + 1, sizeof(int32_t));
    /* pass 1: row lengths */
#pragma omp parallel if (nr > PAR_MIN)
    {
        int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
        for (int64_t c = 0; c < nc; ++c) mark[c] = -1;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nr; ++i) {
            int32_t cnt = 0;
            for (int32_t q = X->rp[i]; q < X->rp[i + 1]; ++q) {
                int32_t k = X->ci[q];
                for (int32_t t = Y->rp[k]; t < Y->rp[k + 1]; ++t)
                    if (mark[Y->ci[t]] != (int32_t)i) { mark[Y->ci[t]] = (int32_t)i; ++cnt; }
            }
            rp[i + 1] = cnt;
        }
        free(mark);
    }
    for (int64_t i = 0; i < nr; ++i) rp[i + 1] += rp[i];
    bsr* Cm = bsr_new(nr, nc, m, p, rp[nr]);
    memcpy(Cm->rp, rp, sizeof(int32_t) * (nr + 1));
    free(rp);
    /* pass 2: sorted columns; pass 3: values through a column -> position map */
#pragma omp parallel if (nr > PAR_MIN)
    {
        int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
        for (int64_t c = 0; c < nc; ++c) mark[c] = -1;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nr; ++i) {
            int32_t nz = Cm->rp[i];
            for (int32_t q = X->rp[i]; q < X->rp[i + 1]; ++q) {
                int32_t k = X->ci[q];
                for (int32_t t = Y->rp[k]; t < Y->rp[k + 1]; ++t)
                    if (mark[Y->ci[t]] != (int32_t)i) { mark[Y->ci[t]] = (int32_t)i; Cm->ci[nz++] = Y->ci[t]; }
            }
            qsort(Cm->ci + Cm->rp[i], Cm->rp[i + 1] - Cm->rp[i], sizeof(int32_t), cmp_i32);
        }
        for (int64_t c = 0; c < nc; ++c) mark[c] = -1;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nr; ++i) {
            for (int32_t q = Cm->rp[i]; q < Cm->rp[i + 1]; ++q) mark[Cm->ci[q]] = q;
            for (int32_t q = X->rp[i]; q < X->rp[i + 1]; ++q) {
                int32_t k = X->ci[q];
                const double* xb = X->v + (int64_t)q * m * n;
                for (int32_t t = Y->rp[k]; t < Y->rp[k + 1]; ++t) {
                    const double* yb = Y->v + (int64_t)t * n * p;
                    double* cb = Cm->v + (int64_t)mark[Y->ci[t]] * m * p;
                    for (int r = 0; r < m; ++r)
                        for (int c = 0; c < p; ++c) {
                            double s = 0.0;
                            for (int l = 0; l < n; ++l) s += xb[r * n + l] * yb[l * p + c];
                            cb[r * p + c] += s;
                        }
                }
            }
        }
        free(mark);
    }
    return Cm;
}

/* R = M^T (block transpose); rows of R list source rows in ascending order. */
static bsr* transpose(const bsr* M) {
    int br = M->br, bc = M->bc;
    bsr* T = bsr_new(M->nc, M->nr, bc, br, M->nnzb);
    for (int64_t q = 0; q < M->nnzb; ++q) T->rp[M->ci[q] + 1]++;
    for (int64_t c = 0; c < M->nc; ++c) T->rp[c + 1] += T->rp[c];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (M->nc > 0 ? M->nc : 1));
    memcpy(fill, T->rp, sizeof(int32_t) * M->nc);
    for (int64_t i = 0; i < M->nr; ++i)
        for (int32_t q = M->rp[i]; q < M->rp[i + 1]; ++q) {
            int32_t pos = fill[M->ci[q]]++;
            T->ci[pos] = (int32_t)i;
            const double* s = M->v + (int64_t)q * br * bc;
            double* d = T->v + (int64_t)pos * br * bc;
            for (int r = 0; r < br; ++r)
                for (int c = 0; c < bc; ++c) d[c * br + r] = s[r * bc + c];
        }
    free(fill);
    return T;
}

/* ------------------------------------------------------------------ dense LU */
/* In-place LU with partial pivoting of the n x n row-major matrix A.  Returns 0, or -1 if a
 * pivot is exactly zero. */
static int lu_factor(int64_t n, double* A, int64_t* piv) {
    for (int64_t k = 0; k < n; ++k) {
        int64_t pr = k;
        double best = fabs(A[k * n + k]);
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); pr = i; }
        piv[k] = pr;
        if (best == 0.0) return -1;
        if (pr != k)
            for (int64_t j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[pr * n + j]; A[pr * n + j] = t; }
#pragma omp parallel for schedule(static) if (n - k > 256)
        for (int64_t i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int64_t j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}
static void lu_solve(int64_t n, const double* LU, const int64_t* piv, double* b) {
    for (int64_t k = 0; k < n; ++k) if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int64_t i = 0; i < n; ++i) { double s = b[i]; for (int64_t j = 0; j < i; ++j) s -= LU[i * n + j] * b[j]; b[i] = s; }
    for (int64_t i = n - 1; i >= 0; --i) { double s = b[i]; for (int64_t j = i + 1; j < n; ++j) s -= LU[i * n + j] * b[j]; b[i] = s / LU[i * n + i]; }
}

/* x = A^-1 b for a dense row-major n x n matrix (A is not modified). */
int orc_dense_solve(int64_t n, const double* A, const double* b, double* x) {
    double* LU = (double*)malloc(sizeof(double) * n * n);
    int64_t* piv = (int64_t*)malloc(sizeof(int64_t) * n);
    memcpy(LU, A, sizeof(double) * n * n);
    int rc = lu_factor(n, LU, piv);
    if (rc == 0) { memcpy(x, b, sizeof(double) * n); lu_solve(n, LU, piv, x); }
    free(LU); free(piv);
    return rc;
}

/* inverse of a small b x b block via LU */
static int small_inverse(int b, const double* A, double* Ai) {
    double LU[64]; int64_t piv[8];
    memcpy(LU, A, sizeof(double) * b * b);
    if (lu_factor(b, LU, piv)) return -1;
    for (int c = 0; c < b; ++c) {
        double e[8] = {0};
        e[c] = 1.0;
        lu_solve(b, LU, piv, e);
        for (int r = 0; r < b; ++r) Ai[r * b + c] = e[r];
    }
    return 0;
}

/* y = M x for generic BSR given as raw arrays (used by tests to check residuals). */
void orc_bsr_spmv(int64_t nr, int64_t nc, int br, int bc, const int32_t* rp, const int32_t* ci,
                  const double* val, const double* x, double* y) {
    bsr M = {nr, nc, br, bc, rp[nr], (int32_t*)rp, (int32_t*)ci, (double*)val};
    bsr_mv(&M, x, y);
}

/* ------------------------------------------------------------------ AMG */
typedef struct {
    double theta;        /* strength threshold at level 0; halved per level */
    int smoother;        /* 0 damped block Jacobi, 1 Chebyshev */
    int cheb_degree;
    double cheb_ratio;   /* lambda_min = lambda_hat / ratio */
    int jacobi_sweeps;
    int coarse_max;      /* stop when the level has at most this many unknowns */
    int max_levels;
    double max_coarse_ratio; /* stop if n_{l+1} > ratio * n_l */
    uint64_t seed;
    int schur_diag;      /* SCR system setup: diagonal used in S^ = C - D d^-1 G:
                            0 the diagonal of A (SCR, SIMPLE), 1 absolute row sums of A (SIMPLEC) */
    int schur_cheb_degree;     /* SCR system: Chebyshev degree of AMG(S^) (0 = cheb_degree; -1 = by the
                                  size of S^: 8 up to 1e6 rows, 12 up to 3e6, 16 above) */
    double schur_cheb_ratio;   /* SCR system: Chebyshev interval ratio of AMG(S^) (0 = cheb_ratio) */
    int amg_type;        /* 0 smoothed aggregation, 1 classical (the paper's settings) */
    double cl_theta;     /* classical strength threshold, 0.5 */
    double trunc;        /* interpolation truncation factor, 0.3 */
    int pmax;            /* interpolation entries per row, 5 */
    int hmis_domain;     /* rows per HMIS domain */
    int gs_domain;       /* rows per hybrid Gauss-Seidel domain */
    int agg_levels;      /* classical: levels coarsened aggressively (two stages), 2 */
    int l1_gs;           /* classical: 1 the l1 hybrid Gauss-Seidel, 0 the plain one */
} amg_opts;

#define MAXLEV 16
typedef struct {
    bsr *A, *P, *R;
    int b, k;
    int32_t* agg;        /* per block row: aggregate id or -1 (isolated) */
    uint8_t* strong;     /* per stored block of A: symmetric strong flag */
    int64_t n_agg;
    double* Dinv;        /* b x b per block row */
    double lam;          /* max abs row sum of D^-1 A */
    double* B;           /* near-null space: (nr*b) x k row-major */
    uint8_t* dead;       /* per coarse dof (n_agg*k) */
    double* Q;           /* tentative prolongator (nr*b) x k row-major */
    uint8_t* func;       /* classical: function (unknown) of each scalar row */
    double* ell;         /* classical, l1 smoother: sign(a_ii) sum of |a_ij| outside i's domain */
} level;

typedef struct {
    int nlev;
    level L[MAXLEV];
    double* LU; int64_t* piv; int64_t ncoarse;
    amg_opts o;
    double* work;        /* scratch vectors */
    int64_t vcycles;
} amg;

/* Strength (squared-Frobenius block norms f_ij, strong iff f_ij^2 >= theta^4 f_ii f_jj,
 * symmetrised by OR).  flags[q] per stored block; iso[i] = no strong off-diagonal neighbour. */
static double block_f(const double* blk, int n) {
    double f = 0.0;
    for (int e = 0; e < n; ++e) f = f + blk[e] * blk[e];
    return f;
}
void orc_strength(int64_t nr, int b, const int32_t* rp, const int32_t* ci, const double* val, double theta,
                  uint8_t* flags, uint8_t* iso) {
    bsr M = {nr, nr, b, b, rp[nr], (int32_t*)rp, (int32_t*)ci, (double*)val};
    int bb = b * b;
    double* fd = (double*)malloc(sizeof(double) * nr);
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i) {
        int32_t q = find_in_row(&M, i, (int32_t)i);
        fd[i] = q >= 0 ? block_f(val + (int64_t)q * bb, bb) : 0.0;
    }
    double th4 = ((theta * theta) * theta) * theta;
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i) {
        iso[i] = 1;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            flags[q] = 0;
            if (j == i) continue;
            double fij = block_f(val + (int64_t)q * bb, bb);
            int s1 = (fij * fij) >= ((th4 * fd[i]) * fd[j]);
            int s2 = 0;
            int32_t t = find_in_row(&M, j, (int32_t)i);
            if (t >= 0) {
                double fji = block_f(val + (int64_t)t * bb, bb);
                s2 = (fji * fji) >= ((th4 * fd[j]) * fd[i]);
            }
            flags[q] = (uint8_t)(s1 || s2);
            if (flags[q]) iso[i] = 0;
        }
    }
    free(fd);
}

/* Priority key of node i at a level: 30 bits of splitmix64 over (seed, level, i), then i. */
static uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}
uint64_t orc_mis_key(uint64_t seed, int level, int64_t i) {
    uint64_t h = sm64(seed ^ ((uint64_t)level << 56) ^ ((uint64_t)i * 0xD1B54A32D192ED03ULL));
    return ((h >> 34) << 32) | (uint64_t)(uint32_t)i;
}

typedef struct { uint64_t key; int32_t i; } keyed;
static int cmp_key_desc(const void* a, const void* b) {
    uint64_t x = ((const keyed*)a)->key, y = ((const keyed*)b)->key;
    return (x < y) - (x > y);
}

/* Distance-2 maximal independent set of the strength graph over non-isolated nodes:
 * sequential greedy in descending key order.  root[i] = 1 for selected nodes. */
void orc_mis2(int64_t nr, const int32_t* rp, const int32_t* ci, const uint8_t* flags, const uint8_t* iso,
              uint64_t seed, int level, uint8_t* root) {
    keyed* order = (keyed*)malloc(sizeof(keyed) * (nr > 0 ? nr : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < nr; ++i) {
        root[i] = 0;
        if (!iso[i]) { order[m].key = orc_mis_key(seed, level, i); order[m].i = (int32_t)i; ++m; }
    }
    qsort(order, m, sizeof(keyed), cmp_key_desc);
    uint8_t* excl = (uint8_t*)calloc(nr > 0 ? nr : 1, 1);
    for (int64_t t = 0; t < m; ++t) {
        int32_t i = order[t].i;
        if (excl[i]) continue;
        root[i] = 1;
        excl[i] = 1;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            if (!flags[q]) continue;
            int32_t j = ci[q];
            excl[j] = 1;
            for (int32_t u = rp[j]; u < rp[j + 1]; ++u) if (flags[u]) excl[ci[u]] = 1;
        }
    }
    free(order); free(excl);
}

/* Aggregates: roots numbered by ascending index; strong neighbours of a root join it;
 * the remaining non-isolated nodes join the aggregate of the strong neighbour, among those
 * that joined in the previous step, with the largest key.  Returns the aggregate count. */
int64_t orc_aggregate(int64_t nr, const int32_t* rp, const int32_t* ci, const uint8_t* flags, const uint8_t* iso,
                      const uint8_t* root, uint64_t seed, int level, int32_t* agg) {
    int64_t na = 0;
    for (int64_t i = 0; i < nr; ++i) agg[i] = root[i] ? (int32_t)na++ : -1;
    uint8_t* step1 = (uint8_t*)calloc(nr > 0 ? nr : 1, 1);
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i) {
        if (iso[i] || root[i]) continue;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
            if (flags[q] && root[ci[q]]) { agg[i] = agg[ci[q]]; step1[i] = 1; break; }
    }
    int lost = 0;
#pragma omp parallel for schedule(static) if (nr > PAR_MIN) reduction(| : lost)
    for (int64_t i = 0; i < nr; ++i) {
        if (iso[i] || agg[i] >= 0 || step1[i]) continue;
        uint64_t best = 0; int32_t bj = -1;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            if (!flags[q] || !step1[j]) continue;
            uint64_t kj = orc_mis_key(seed, level, j);
            if (bj < 0 || kj > best) { best = kj; bj = j; }
        }
        if (bj < 0) { lost = 1; continue; }      /* cannot happen for a maximal set */
        agg[i] = agg[bj];                          /* bj joined in the previous step: final */
    }
    free(step1);
    return lost ? -1 : na;
}

/* Tentative prolongator by Gram-Schmidt (two modified-GS passes) of the near-null space
 * restricted to each aggregate (its nodes in ascending order).  Column j is dead when its
 * remainder is <= 1e-10 of its own norm: q_j = 0, R_jj = 0.  Q gives P_tent (b x k block
 * per fine node), R gives the coarse near-null space (k x k block per aggregate). */
static void tentative(int64_t nr, int b, int k, const int32_t* agg, int64_t na, const double* B,
                      double* Q /* nr*b x k */, double* Bc /* na*k x k */, uint8_t* dead /* na*k */) {
    int64_t* cnt = (int64_t*)calloc(na + 1, sizeof(int64_t));
    for (int64_t i = 0; i < nr; ++i) if (agg[i] >= 0) cnt[agg[i] + 1]++;
    for (int64_t a = 0; a < na; ++a) cnt[a + 1] += cnt[a];
    int32_t* mem = (int32_t*)malloc(sizeof(int32_t) * (cnt[na] > 0 ? cnt[na] : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (na > 0 ? na : 1));
    memcpy(fill, cnt, sizeof(int64_t) * na);
    for (int64_t i = 0; i < nr; ++i) if (agg[i] >= 0) mem[fill[agg[i]]++] = (int32_t)i;
    memset(Q, 0, sizeof(double) * nr * b * k);
    memset(Bc, 0, sizeof(double) * na * k * k);
#pragma omp parallel for schedule(dynamic, 64) if (na > 256)
    for (int64_t a = 0; a < na; ++a) {
        int64_t nn = cnt[a + 1] - cnt[a];
        int64_t rows = nn * b;
        double* W = (double*)malloc(sizeof(double) * rows * k);   /* columns of B on the aggregate */
        for (int64_t t = 0; t < nn; ++t)
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < k; ++c) W[(t * b + r) * k + c] = B[((int64_t)mem[cnt[a] + t] * b + r) * k + c];
        double* Rk = Bc + a * k * k;
        for (int j = 0; j < k; ++j) {
            double nb = 0.0;
            for (int64_t r = 0; r < rows; ++r) nb += W[r * k + j] * W[r * k + j];
            nb = sqrt(nb);
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i < j; ++i) {
                    if (dead[a * k + i]) continue;
                    double c = 0.0;
                    for (int64_t r = 0; r < rows; ++r) c += W[r * k + i] * W[r * k + j];
                    for (int64_t r = 0; r < rows; ++r) W[r * k + j] -= c * W[r * k + i];
                    Rk[i * k + j] += c;
                }
            double nv = 0.0;
            for (int64_t r = 0; r < rows; ++r) nv += W[r * k + j] * W[r * k + j];
            nv = sqrt(nv);
            if (nb == 0.0 || nv <= 1e-10 * nb) {
                dead[a * k + j] = 1;
                for (int64_t r = 0; r < rows; ++r) W[r * k + j] = 0.0;
                Rk[j * k + j] = 0.0;
            } else {
                dead[a * k + j] = 0;
                for (int64_t r = 0; r < rows; ++r) W[r * k + j] /= nv;
                Rk[j * k + j] = nv;
            }
        }
        for (int64_t t = 0; t < nn; ++t)
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < k; ++c) Q[((int64_t)mem[cnt[a] + t] * b + r) * k + c] = W[(t * b + r) * k + c];
        free(W);
    }
    free(cnt); free(mem); free(fill);
}

static void level_free(level* L) {
    bsr_free(L->A); bsr_free(L->P); bsr_free(L->R);
    free(L->agg); free(L->strong); free(L->Dinv); free(L->B); free(L->dead); free(L->Q); free(L->func);
    free(L->ell);
}

/* D^-1 (block diagonal inverse) and lambda_hat = max abs row sum of D^-1 A */
static int level_diag(level* L) {
    const bsr* A = L->A;
    int b = L->b, bb = b * b;
    L->Dinv = (double*)malloc(sizeof(double) * A->nr * bb);
    double lam = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) if (A->nr > PAR_MIN) reduction(max : lam) reduction(| : bad)
    for (int64_t i = 0; i < A->nr; ++i) {
        int32_t q = find_in_row(A, i, (int32_t)i);
        if (q < 0 || small_inverse(b, A->v + (int64_t)q * bb, L->Dinv + i * bb)) { bad = 1; continue; }
        double rs[8] = {0};
        for (int32_t t = A->rp[i]; t < A->rp[i + 1]; ++t) {
            const double* blk = A->v + (int64_t)t * bb;
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < b; ++c) {
                    double s = 0.0;
                    for (int l = 0; l < b; ++l) s += L->Dinv[i * bb + r * b + l] * blk[l * b + c];
                    rs[r] += fabs(s);
                }
        }
        for (int r = 0; r < b; ++r) if (rs[r] > lam) lam = rs[r];
    }
    if (bad) return -1;
    L->lam = lam;
    return 0;
}

/* Smoothed prolongator P = (I - omega D^-1 A) P_tent, omega = 4/(3 lambda_hat); rows of
 * isolated nodes are empty; pattern = aggregates of the non-isolated structural neighbours. */
static bsr* smooth_prolongator(const level* L, const double* Q) {
    const bsr* A = L->A;
    int b = L->b, k = L->k, bb = b * b;
    double omega = 4.0 / (3.0 * L->lam);
    int64_t nr = A->nr;
    /* pattern */
    int32_t* rp = (int32_t*)calloc(nr + 1, sizeof(int32_t));
    int64_t cap = nr * 4 + 16, nnz = 0;
    int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * cap);
    for (int64_t i = 0; i < nr; ++i) {
        int64_t start = nnz;
        if (L->agg[i] >= 0)
            for (int32_t q = A->rp[i]; q < A->rp[i + 1]; ++q) {
                int32_t a = L->agg[A->ci[q]];
                if (a < 0) continue;
                int dup = 0;
                for (int64_t t = start; t < nnz; ++t) if (ci[t] == a) { dup = 1; break; }
                if (dup) continue;
                if (nnz == cap) { cap *= 2; ci = (int32_t*)realloc(ci, sizeof(int32_t) * cap); }
                ci[nnz++] = a;
            }
        qsort(ci + start, nnz - start, sizeof(int32_t), cmp_i32);
        rp[i + 1] = (int32_t)nnz;
    }
    bsr* P = bsr_new(nr, L->n_agg, b, k, nnz);
    memcpy(P->rp, rp, sizeof(int32_t) * (nr + 1));
    memcpy(P->ci, ci, sizeof(int32_t) * nnz);
    free(rp); free(ci);
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i) {
        if (L->agg[i] < 0) continue;
        const double* Di = L->Dinv + i * bb;
        for (int32_t q = A->rp[i]; q < A->rp[i + 1]; ++q) {
            int32_t j = A->ci[q];
            if (L->agg[j] < 0) continue;
            double T[64];     /* D_i^-1 A_ij */
            const double* blk = A->v + (int64_t)q * bb;
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < b; ++c) {
                    double s = 0.0;
                    for (int l = 0; l < b; ++l) s += Di[r * b + l] * blk[l * b + c];
                    T[r * b + c] = s;
                }
            int32_t pos = find_in_row(P, i, L->agg[j]);
            double* pb = P->v + (int64_t)pos * b * k;
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < k; ++c) {
                    double s = 0.0;
                    for (int l = 0; l < b; ++l) s += T[r * b + l] * Q[((int64_t)j * b + l) * k + c];
                    pb[r * k + c] -= omega * s;
                }
        }
        int32_t pos = find_in_row(P, i, L->agg[i]);
        double* pb = P->v + (int64_t)pos * b * k;
        for (int r = 0; r < b; ++r)
            for (int c = 0; c < k; ++c) pb[r * k + c] += Q[(i * b + r) * k + c];
    }
    return P;
}

void orc_amg_free(amg* h) {
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) level_free(&h->L[l]);
    free(h->LU); free(h->piv); free(h->work);
    free(h);
}

/* The value-dependent part of level l, given its aggregates: D^-1 and lambda_hat, the tentative
 * prolongator (with the coarse near-null space and dead coarse dofs), the smoothed prolongator,
 * R = P^T and the Galerkin product A_{l+1} = R A P (dead coarse dofs get a unit diagonal).
 * Replaces whatever these fields held. */
static int level_numeric(amg* h, int l) {
    level* L = &h->L[l];
    level* N = &h->L[l + 1];
    int64_t nr = L->A->nr;
    free(L->Dinv); L->Dinv = NULL;
    if (level_diag(L)) return -1;
    free(L->Q); free(N->B); free(L->dead);
    bsr_free(L->P); bsr_free(L->R); bsr_free(N->A);
    double* Q = (double*)malloc(sizeof(double) * nr * L->b * L->k);
    N->b = L->k; N->k = L->k;
    N->B = (double*)malloc(sizeof(double) * L->n_agg * L->k * L->k);
    L->dead = (uint8_t*)calloc(L->n_agg * L->k, 1);
    tentative(nr, L->b, L->k, L->agg, L->n_agg, L->B, Q, N->B, L->dead);
    L->P = smooth_prolongator(L, Q);
    L->Q = Q;
    L->R = transpose(L->P);
    bsr* AP = spgemm(L->A, L->P);
    N->A = spgemm(L->R, AP);
    bsr_free(AP);
    for (int64_t a = 0; a < L->n_agg; ++a)
        for (int c = 0; c < L->k; ++c)
            if (L->dead[a * L->k + c]) {
                int32_t q = find_in_row(N->A, a, (int32_t)a);
                N->A->v[(int64_t)q * L->k * L->k + c * L->k + c] = 1.0;
            }
    return 0;
}

/* Coarsest level: dense LU of A_c. */
static int coarse_factor(amg* h) {
    level* Lc = &h->L[h->nlev - 1];
    int64_t nc = Lc->A->nr * Lc->b;
    h->ncoarse = nc;
    free(h->LU); free(h->piv);
    h->LU = (double*)calloc((size_t)nc * nc, sizeof(double));
    h->piv = (int64_t*)malloc(sizeof(int64_t) * (nc > 0 ? nc : 1));
    int b = Lc->b;
    for (int64_t i = 0; i < Lc->A->nr; ++i)
        for (int32_t q = Lc->A->rp[i]; q < Lc->A->rp[i + 1]; ++q)
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < b; ++c)
                    h->LU[(i * b + r) * nc + (int64_t)Lc->A->ci[q] * b + c] = Lc->A->v[(int64_t)q * b * b + r * b + c];
    return lu_factor(nc, h->LU, h->piv);
}

/* ------------------------------------------------------------------ classical AMG
 * The paper's preconditioner settings (Sec. 5.2, table of AMG settings): classical strength with
 * threshold 0.5, HMIS coarsening, extended+i interpolation truncated at 0.3 with at most 5
 * entries per row, hybrid Gauss-Seidel smoothing, V-cycle.  Restated here:
 *
 * Strength (scalar rows; "functions" f(i) give the unknown approach for systems: only couplings
 * between unknowns of the same function count).  With s = sign(a_ii) (+1 for a_ii = 0) and
 * m_i = max over j != i, f(j) = f(i) of -s a_ij, row i depends strongly on j iff m_i > 0 and
 * -s a_ij >= theta m_i.  S_i: the points i depends on; S^T_i: the points that depend on i.
 *
 * HMIS (De Sterck, Yang and Heys): rows are cut into domains of `dom` consecutive rows (the
 * processor domains of a distributed run).  In each domain, the first pass of Ruge-Stueben
 * coarsening on the strength graph restricted to the domain: measure lambda_i = number of domain
 * points depending on i; points with no dependency either way inside the domain are F; then
 * repeatedly the undecided point of largest measure (lowest index on ties) becomes C, the
 * undecided domain points depending on it become F, the undecided domain points it depends on
 * lose one unit of measure, and for each new F point the undecided domain points it depends on
 * gain one.  The C points of this pass whose strong connections (both directions) all stay in
 * their domain start PMIS over the whole graph: measure w_i = |S^T_i| + u_i with u_i uniform in
 * [0, 1) from splitmix64 of (seed, level, i); every other point with |S^T_i| = 0 is F and the
 * rest undecided; then repeatedly every undecided point depending on a C point of the previous
 * round becomes F, and every undecided point whose w beats that of every undecided strong
 * neighbour (either direction; ties to the lower index) becomes C.
 *
 * Extended+i interpolation (De Sterck, Falgout, Nolting and Yang).  For an F point i: C^_i = the
 * C points of S_i and the C points of S_k for every F point k of S_i.  For such a k, with
 * a'_kl = a_kl where a_kl and a_kk have opposite signs (else 0), den_k = sum of a'_kl over
 * l in C^_i and l = i.  Then, running over row i (same function, j != i, ascending columns):
 * a_ij for j in C^_i goes to num_j; for a strong F neighbour k with den_k != 0 the terms
 * a_ik a'_kl / den_k (row k ascending, l in C^_i or l = i) go to num_l, or to the diagonal when
 * l = i; every other coupling (weak, or den_k = 0) is added to the diagonal a~_ii, which starts at
 * a_ii.  w_ij = -num_j / a~_ii.  Truncation: entries below trunc * max |w| are dropped, then all
 * but the pmax largest in magnitude (ties to the lower column), and the kept entries are scaled
 * so that the row keeps its sum.  C points interpolate themselves with weight 1.
 *
 * Aggressive coarsening (the first agg_levels levels): HMIS on S gives first-stage C points; HMIS
 * again, on the graph in which C point i depends on C point j when a path of one or two strong
 * dependencies leads from i to j, keeps a subset of them as the level's C points.  Interpolation in
 * two stages of extended+i: P1 from the fine points onto the first-stage C points (on A), P2 from
 * those onto the kept ones (on A1 = P1^T A P1 with its own strength), P = P1 P2, each truncated as
 * above.
 *
 * Hybrid Gauss-Seidel (Baker, Falgout, Kolev and Yang): Gauss-Seidel inside domains of `gs_dom`
 * consecutive rows, Jacobi between them: x_i = (b_i - sum_{j != i} a_ij x~_j) / a_ii with x~_j
 * the new value for j earlier in the same domain (forward sweep: j < i; backward: j > i) and the
 * previous iterate otherwise.  The l1 form of the same paper adds to the splitting's diagonal
 * d_i = s sum |a_ij| over the columns j outside i's domain (s = sign(a_ii)): the sweep is
 * x = x_old + M^-1 (b - A x_old) with M = (a_ii + d_i) on the diagonal and the in-domain lower
 * (forward) or upper (backward) part of A, that is x_i = (b_i - sum_{j != i} a_ij x~_j + d_i x_old_i)
 * / (a_ii + d_i); for symmetric positive definite A it converges whatever the domains, where the
 * plain sweep may diverge once D^-1 A has eigenvalues above 2.  V-cycle: one forward sweep from
 * zero, coarse-grid correction, one backward sweep (a symmetric cycle for symmetric A).
 */
static int opposite(double a, double d) { return (a > 0.0 && d < 0.0) || (a < 0.0 && d > 0.0); }

void orc_cl_strength(int64_t nr, const int32_t* rp, const int32_t* ci, const double* val, const uint8_t* func,
                     double theta, uint8_t* S) {
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i) {
        double aii = 0.0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
            if (ci[q] == i) aii = val[q];
        double sg = aii < 0.0 ? -1.0 : 1.0;
        int have = 0;
        double m = 0.0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            if (j == i || func[j] != func[i]) continue;
            double v = -sg * val[q];
            if (!have || v > m) { m = v; have = 1; }
        }
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            int32_t j = ci[q];
            S[q] = 0;
            if (j == i || func[j] != func[i] || !have || !(m > 0.0)) continue;
            S[q] = (uint8_t)(-sg * val[q] >= theta * m);
        }
    }
}

/* position of (j, i) for every stored (i, j); -1 if the pattern lacks it */
static int32_t* transpose_map(int64_t nr, const int32_t* rp, const int32_t* ci) {
    int32_t* t = (int32_t*)malloc(sizeof(int32_t) * (rp[nr] > 0 ? rp[nr] : 1));
    bsr M = {nr, nr, 1, 1, rp[nr], (int32_t*)rp, (int32_t*)ci, NULL};
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i)
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) t[q] = find_in_row(&M, ci[q], (int32_t)i);
    return t;
}

double orc_cl_uniform(uint64_t seed, int level, int64_t i) {
    uint64_t h = sm64(seed ^ ((uint64_t)level << 56) ^ ((uint64_t)i * 0x9E6C63D0676A9A99ULL));
    return (double)(h >> 11) * 0x1.0p-53;
}

/* cf[i] = 1 (C) or -1 (F); first[i] = the first pass's decision (1 C, -1 F).  Returns 0, or -1
 * if the pattern is not structurally symmetric. */
int orc_cl_hmis(int64_t nr, const int32_t* rp, const int32_t* ci, const uint8_t* S, int dom, uint64_t seed,
                int level, int8_t* cf, int8_t* first) {
    int32_t* tm = transpose_map(nr, rp, ci);
    for (int64_t q = 0; q < rp[nr]; ++q)
        if (tm[q] < 0) { free(tm); return -1; }
    /* ST[q] for q = (i, j): j depends on i */
    uint8_t* ST = (uint8_t*)malloc(rp[nr] > 0 ? rp[nr] : 1);
    for (int64_t q = 0; q < rp[nr]; ++q) ST[q] = S[tm[q]];
    free(tm);
    int32_t* lam = (int32_t*)malloc(sizeof(int32_t) * (nr > 0 ? nr : 1));
    int8_t* st = (int8_t*)malloc(nr > 0 ? nr : 1);              /* 0 undecided, 1 C, 2 F */
    int32_t* newf = (int32_t*)malloc(sizeof(int32_t) * (nr > 0 ? nr : 1));
    for (int64_t d0 = 0; d0 < nr; d0 += dom) {
        int64_t d1 = d0 + dom < nr ? d0 + dom : nr;
        for (int64_t i = d0; i < d1; ++i) {
            int32_t l = 0, dep = 0;
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
                int32_t j = ci[q];
                if (j < d0 || j >= d1) continue;
                l += ST[q];
                dep += S[q];
            }
            lam[i] = l;
            st[i] = (l == 0 && dep == 0) ? 2 : 0;
        }
        for (;;) {
            int64_t c = -1;
            for (int64_t i = d0; i < d1; ++i)
                if (st[i] == 0 && (c < 0 || lam[i] > lam[c])) c = i;
            if (c < 0) break;
            st[c] = 1;
            int64_t nf = 0;
            for (int32_t q = rp[c]; q < rp[c + 1]; ++q) {
                int32_t j = ci[q];
                if (j >= d0 && j < d1 && st[j] == 0 && ST[q]) { st[j] = 2; newf[nf++] = j; }
            }
            for (int32_t q = rp[c]; q < rp[c + 1]; ++q) {
                int32_t j = ci[q];
                if (j >= d0 && j < d1 && st[j] == 0 && S[q]) lam[j] -= 1;
            }
            for (int64_t t = 0; t < nf; ++t) {
                int32_t j = newf[t];
                for (int32_t q = rp[j]; q < rp[j + 1]; ++q) {
                    int32_t k = ci[q];
                    if (k >= d0 && k < d1 && st[k] == 0 && S[q]) lam[k] += 1;
                }
            }
        }
    }
    for (int64_t i = 0; i < nr; ++i) first[i] = st[i] == 1 ? 1 : -1;
    /* PMIS, started from the interior C points of the first pass */
    double* w = (double*)malloc(sizeof(double) * (nr > 0 ? nr : 1));
    uint8_t* isnew = (uint8_t*)malloc(nr > 0 ? nr : 1);
    int8_t* nx = (int8_t*)malloc(nr > 0 ? nr : 1);
    for (int64_t i = 0; i < nr; ++i) {
        int64_t dm = i / dom;
        int interior = 1;
        int32_t nst = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            nst += ST[q];
            if ((S[q] || ST[q]) && ci[q] / dom != dm) interior = 0;
        }
        w[i] = (double)nst + orc_cl_uniform(seed, level, i);
        if (first[i] == 1 && interior) st[i] = 1;
        else st[i] = nst == 0 ? 2 : 0;
        isnew[i] = st[i] == 1;
    }
    for (;;) {
        for (int64_t i = 0; i < nr; ++i) {
            nx[i] = st[i];
            if (st[i] != 0) continue;
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
                if (S[q] && isnew[ci[q]]) { nx[i] = 2; break; }
        }
        int64_t und = 0;
        for (int64_t i = 0; i < nr; ++i) { st[i] = nx[i]; und += st[i] == 0; isnew[i] = 0; }
        if (und == 0) break;
        for (int64_t i = 0; i < nr; ++i) {
            if (st[i] != 0) continue;
            int best = 1;
            for (int32_t q = rp[i]; q < rp[i + 1] && best; ++q) {
                int32_t j = ci[q];
                if (j == i || st[j] != 0 || !(S[q] || ST[q])) continue;
                if (!(w[i] > w[j] || (w[i] == w[j] && i < j))) best = 0;
            }
            if (best) isnew[i] = 1;
        }
        for (int64_t i = 0; i < nr; ++i)
            if (isnew[i]) st[i] = 1;
    }
    for (int64_t i = 0; i < nr; ++i) cf[i] = st[i] == 1 ? 1 : -1;
    free(ST); free(lam); free(st); free(newf); free(w); free(isnew); free(nx);
    return 0;
}

static int cmp_i32_asc(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}
static int64_t find_sorted(const int32_t* v, int64_t n, int32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (v[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && v[lo] == key) ? lo : -1;
}

/* One row of extended+i interpolation (F point i).  hat: sorted C^_i (fine indices), m entries;
 * w: m weights out.  Returns 0, or 1 if the modified diagonal is zero (empty row). */
static int extpi_row(const int32_t* rp, const int32_t* ci, const double* val, const uint8_t* func, const uint8_t* S,
                     const int32_t* cidx, int64_t i, const int32_t* hat, int64_t m, double* w) {
    double diag = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        if (ci[q] == i) diag = val[q];
    for (int64_t t = 0; t < m; ++t) w[t] = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        int32_t n = ci[q];
        if (n == i || func[n] != func[i]) continue;
        int64_t p = find_sorted(hat, m, n);
        if (p >= 0) { w[p] = w[p] + val[q]; continue; }
        if (S[q] && cidx[n] < 0) {
            double ann = 0.0, den = 0.0;
            for (int32_t r = rp[n]; r < rp[n + 1]; ++r)
                if (ci[r] == n) ann = val[r];
            for (int32_t r = rp[n]; r < rp[n + 1]; ++r) {
                int32_t l = ci[r];
                if ((l == i || find_sorted(hat, m, l) >= 0) && opposite(val[r], ann)) den = den + val[r];
            }
            if (den == 0.0) { diag = diag + val[q]; continue; }
            for (int32_t r = rp[n]; r < rp[n + 1]; ++r) {
                int32_t l = ci[r];
                if (!opposite(val[r], ann)) continue;
                double t = (val[q] * val[r]) / den;
                if (l == i) diag = diag + t;
                else {
                    int64_t pl = find_sorted(hat, m, l);
                    if (pl >= 0) w[pl] = w[pl] + t;
                }
            }
            continue;
        }
        diag = diag + val[q];
    }
    if (diag == 0.0) return 1;
    for (int64_t t = 0; t < m; ++t) w[t] = -w[t] / diag;
    return 0;
}

typedef struct { double a; int32_t c; } wcol;
static int cmp_wcol(const void* x, const void* y) {
    const wcol* p = (const wcol*)x;
    const wcol* q = (const wcol*)y;
    if (p->a != q->a) return p->a > q->a ? -1 : 1;
    return (p->c > q->c) - (p->c < q->c);
}

/* Truncation of one row (columns ascending): keep |w| >= trunc * max |w| (and w != 0), then the
 * pmax largest, then scale the kept entries to the row's original sum.  Compacts in place and
 * returns the kept count. */
static int64_t truncate_row(int32_t* col, double* w, int64_t m, double trunc, int pmax) {
    double mx = 0.0, all = 0.0;
    for (int64_t t = 0; t < m; ++t) {
        all = all + w[t];
        if (fabs(w[t]) > mx) mx = fabs(w[t]);
    }
    int64_t k = 0;
    for (int64_t t = 0; t < m; ++t)
        if (w[t] != 0.0 && fabs(w[t]) >= trunc * mx) { col[k] = col[t]; w[k] = w[t]; ++k; }
    if (pmax > 0 && k > pmax) {
        wcol* tmp = (wcol*)malloc(sizeof(wcol) * k);
        for (int64_t t = 0; t < k; ++t) { tmp[t].a = fabs(w[t]); tmp[t].c = col[t]; }
        qsort(tmp, k, sizeof(wcol), cmp_wcol);
        /* keep the first pmax of the magnitude order, in ascending columns */
        int32_t* keep = (int32_t*)malloc(sizeof(int32_t) * pmax);
        for (int t = 0; t < pmax; ++t) keep[t] = tmp[t].c;
        qsort(keep, pmax, sizeof(int32_t), cmp_i32_asc);
        int64_t k2 = 0;
        for (int64_t t = 0; t < k; ++t)
            if (find_sorted(keep, pmax, col[t]) >= 0) { col[k2] = col[t]; w[k2] = w[t]; ++k2; }
        k = k2;
        free(tmp); free(keep);
    }
    double kept = 0.0;
    for (int64_t t = 0; t < k; ++t) kept = kept + w[t];
    if (kept != 0.0) {
        double sc = all / kept;
        for (int64_t t = 0; t < k; ++t) w[t] = w[t] * sc;
    }
    return k;
}

/* Extended+i interpolation P (nr x nc, 1x1 blocks) from the C/F split (cidx: coarse index or -1). */
static bsr* extpi(int64_t nr, int64_t nc, const int32_t* rp, const int32_t* ci, const double* val, const uint8_t* func,
                  const uint8_t* S, const int32_t* cidx, double trunc, int pmax) {
    int32_t** rc = (int32_t**)calloc(nr > 0 ? nr : 1, sizeof(int32_t*));
    double** rw = (double**)calloc(nr > 0 ? nr : 1, sizeof(double*));
    int64_t* rn = (int64_t*)calloc(nr > 0 ? nr : 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256) if (nr > PAR_MIN)
    for (int64_t i = 0; i < nr; ++i) {
        if (cidx[i] >= 0) {
            rc[i] = (int32_t*)malloc(sizeof(int32_t)); rw[i] = (double*)malloc(sizeof(double));
            rc[i][0] = cidx[i]; rw[i][0] = 1.0; rn[i] = 1;
            continue;
        }
        int64_t cap = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            if (!S[q]) continue;
            int32_t j = ci[q];
            if (cidx[j] >= 0) ++cap;
            else cap += rp[j + 1] - rp[j];
        }
        int32_t* hat = (int32_t*)malloc(sizeof(int32_t) * (cap > 0 ? cap : 1));
        int64_t m = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            if (!S[q]) continue;
            int32_t j = ci[q];
            if (cidx[j] >= 0) { hat[m++] = j; continue; }
            for (int32_t r = rp[j]; r < rp[j + 1]; ++r)
                if (S[r] && cidx[ci[r]] >= 0) hat[m++] = ci[r];
        }
        qsort(hat, m, sizeof(int32_t), cmp_i32_asc);
        int64_t u = 0;
        for (int64_t t = 0; t < m; ++t)
            if (u == 0 || hat[t] != hat[u - 1]) hat[u++] = hat[t];
        m = u;
        double* w = (double*)malloc(sizeof(double) * (m > 0 ? m : 1));
        if (m == 0 || extpi_row(rp, ci, val, func, S, cidx, i, hat, m, w)) m = 0;
        for (int64_t t = 0; t < m; ++t) hat[t] = cidx[hat[t]];
        rn[i] = truncate_row(hat, w, m, trunc, pmax);
        rc[i] = hat; rw[i] = w;
    }
    int64_t nnz = 0;
    for (int64_t i = 0; i < nr; ++i) nnz += rn[i];
    bsr* P = bsr_new(nr, nc, 1, 1, nnz);
    for (int64_t i = 0; i < nr; ++i) {
        P->rp[i + 1] = P->rp[i] + (int32_t)rn[i];
        memcpy(P->ci + P->rp[i], rc[i], sizeof(int32_t) * rn[i]);
        memcpy(P->v + P->rp[i], rw[i], sizeof(double) * rn[i]);
        free(rc[i]); free(rw[i]);
    }
    free(rc); free(rw); free(rn);
    return P;
}

/* test entry: P of a given split; prp (nr + 1) always, pci/pv (nnz) when not NULL; returns nnz */
int64_t orc_cl_extpi(int64_t nr, const int32_t* rp, const int32_t* ci, const double* val, const uint8_t* func,
                     const uint8_t* S, const int8_t* cf, double trunc, int pmax, int32_t* prp, int32_t* pci,
                     double* pv) {
    int32_t* cidx = (int32_t*)malloc(sizeof(int32_t) * (nr > 0 ? nr : 1));
    int64_t nc = 0;
    for (int64_t i = 0; i < nr; ++i) cidx[i] = cf[i] == 1 ? (int32_t)nc++ : -1;
    bsr* P = extpi(nr, nc, rp, ci, val, func, S, cidx, trunc, pmax);
    memcpy(prp, P->rp, sizeof(int32_t) * (nr + 1));
    if (pci) memcpy(pci, P->ci, sizeof(int32_t) * P->nnzb);
    if (pv) memcpy(pv, P->v, sizeof(double) * P->nnzb);
    int64_t nnz = P->nnzb;
    bsr_free(P); free(cidx);
    return nnz;
}

/* One hybrid Gauss-Seidel sweep (x out; xold the previous iterate, NULL = zero). */
static void hybrid_gs(const bsr* A, const double* Dinv, const double* ell, int dom, int backward, const double* b,
                      const double* xold, double* x) {
    int64_t nr = A->nr;
    int64_t nd = (nr + dom - 1) / dom;
#pragma omp parallel for schedule(static) if (nr > PAR_MIN)
    for (int64_t d = 0; d < nd; ++d) {
        int64_t lo = d * dom, hi = lo + dom < nr ? lo + dom : nr;
        for (int64_t t = 0; t < hi - lo; ++t) {
            int64_t i = backward ? hi - 1 - t : lo + t;
            double s = 0.0;
            for (int32_t q = A->rp[i]; q < A->rp[i + 1]; ++q) {
                int64_t j = A->ci[q];
                if (j == i) continue;
                int fresh = j >= lo && j < hi && (backward ? j > i : j < i);
                double xj = fresh ? x[j] : (xold ? xold[j] : 0.0);
                s = s + A->v[q] * xj;
            }
            double t = b[i] - s;
            if (ell && xold) t = t + ell[i] * xold[i];
            x[i] = t * Dinv[i];
        }
    }
}

/* The l1 term of every row (ell) and the inverse of the l1 diagonal a_ii + ell_i (Dinv). */
static void l1_diag(const bsr* A, int dom, double* ell, double* Dinv) {
    for (int64_t i = 0; i < A->nr; ++i) {
        double aii = 0.0, e = 0.0;
        for (int32_t q = A->rp[i]; q < A->rp[i + 1]; ++q) {
            int64_t j = A->ci[q];
            if (j == i) aii = A->v[q];
            else if (j / dom != i / dom) e = e + fabs(A->v[q]);
        }
        ell[i] = aii < 0.0 ? -e : e;
        Dinv[i] = 1.0 / (aii + ell[i]);
    }
}

/* test entry: one hybrid Gauss-Seidel sweep (l1 form when l1 != 0) */
void orc_cl_gs(int64_t nr, const int32_t* rp, const int32_t* ci, const double* val, int dom, int backward, int l1,
               const double* b, const double* xold, double* x) {
    bsr A = {nr, nr, 1, 1, rp[nr], (int32_t*)rp, (int32_t*)ci, (double*)val};
    double* Dinv = (double*)malloc(sizeof(double) * (nr > 0 ? nr : 1));
    double* ell = (double*)malloc(sizeof(double) * (nr > 0 ? nr : 1));
    if (l1) {
        l1_diag(&A, dom, ell, Dinv);
    } else {
        for (int64_t i = 0; i < nr; ++i) {
            Dinv[i] = 0.0;
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
                if (ci[q] == i) Dinv[i] = 1.0 / val[q];
        }
    }
    hybrid_gs(&A, Dinv, l1 ? ell : NULL, dom, backward, b, xold, x);
    free(Dinv);
    free(ell);
}

/* the scalar matrix of a b x b BSR matrix (row b*i + r, columns in order) and the function of
 * each scalar row (r) */
static bsr* to_scalar(const bsr* A, uint8_t** func) {
    int b = A->br;
    bsr* S = bsr_new(A->nr * b, A->nc * b, 1, 1, A->nnzb * b * b);
    *func = (uint8_t*)malloc(A->nr * b > 0 ? A->nr * b : 1);
    int64_t p = 0;
    for (int64_t i = 0; i < A->nr; ++i)
        for (int r = 0; r < b; ++r) {
            int64_t row = i * b + r;
            (*func)[row] = (uint8_t)r;
            for (int32_t q = A->rp[i]; q < A->rp[i + 1]; ++q)
                for (int c = 0; c < b; ++c) {
                    S->ci[p] = A->ci[q] * b + c;
                    S->v[p] = A->v[(int64_t)q * b * b + r * b + c];
                    ++p;
                }
            S->rp[row + 1] = (int32_t)p;
        }
    return S;
}

/* Aggressive coarsening, second stage: the graph on the first-stage C points (c1[i] = index among
 * them, -1 for F points) in which C point i depends on C point j when j is reached from i by a
 * path of one or two strong dependencies (S_i, or S_k for k in S_i).  Returned as a structurally
 * symmetric pattern (the union of the edges and their reverses, columns ascending) with a flag per
 * entry for the edges themselves. */
static void second_stage_graph(int64_t n, const int32_t* rp, const int32_t* ci, const uint8_t* S, const int32_t* c1,
                               int64_t n1, int32_t** grp, int32_t** gci, uint8_t** gS) {
    int32_t** out = (int32_t**)calloc(n1 > 0 ? n1 : 1, sizeof(int32_t*));
    int64_t* no = (int64_t*)calloc(n1 > 0 ? n1 : 1, sizeof(int64_t));
    int64_t* nin = (int64_t*)calloc(n1 > 0 ? n1 : 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (c1[i] < 0) continue;
        int64_t cap = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
            if (S[q]) cap += 1 + (rp[ci[q] + 1] - rp[ci[q]]);
        int32_t* e = (int32_t*)malloc(sizeof(int32_t) * (cap > 0 ? cap : 1));
        int64_t m = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            if (!S[q]) continue;
            int32_t k = ci[q];
            if (c1[k] >= 0 && k != i) e[m++] = c1[k];
            for (int32_t r = rp[k]; r < rp[k + 1]; ++r)
                if (S[r] && c1[ci[r]] >= 0 && ci[r] != i) e[m++] = c1[ci[r]];
        }
        qsort(e, m, sizeof(int32_t), cmp_i32_asc);
        int64_t u = 0;
        for (int64_t t2 = 0; t2 < m; ++t2)
            if (u == 0 || e[t2] != e[u - 1]) e[u++] = e[t2];
        out[c1[i]] = e;
        no[c1[i]] = u;
    }
    for (int64_t a = 0; a < n1; ++a)
        for (int64_t t2 = 0; t2 < no[a]; ++t2) nin[out[a][t2]]++;
    int32_t** in = (int32_t**)calloc(n1 > 0 ? n1 : 1, sizeof(int32_t*));
    for (int64_t a = 0; a < n1; ++a) { in[a] = (int32_t*)malloc(sizeof(int32_t) * (nin[a] > 0 ? nin[a] : 1)); nin[a] = 0; }
    for (int64_t a = 0; a < n1; ++a)
        for (int64_t t2 = 0; t2 < no[a]; ++t2) { int32_t b = out[a][t2]; in[b][nin[b]++] = (int32_t)a; }
    int32_t* rp2 = (int32_t*)calloc(n1 + 1, sizeof(int32_t));
    int64_t tot = 0;
    for (int64_t a = 0; a < n1; ++a) tot += no[a] + nin[a];
    int32_t* ci2 = (int32_t*)malloc(sizeof(int32_t) * (tot > 0 ? tot : 1));
    uint8_t* f2 = (uint8_t*)malloc(tot > 0 ? tot : 1);
    int64_t p = 0;
    for (int64_t a = 0; a < n1; ++a) {
        /* merge the sorted out-list with the (ascending) in-list */
        int64_t x = 0, y = 0;
        while (x < no[a] || y < nin[a]) {
            int32_t cx = x < no[a] ? out[a][x] : INT32_MAX, cy = y < nin[a] ? in[a][y] : INT32_MAX;
            int32_t c = cx < cy ? cx : cy;
            ci2[p] = c;
            f2[p] = cx == c;
            if (cx == c) ++x;
            if (cy == c) ++y;
            ++p;
        }
        rp2[a + 1] = (int32_t)p;
        free(out[a]); free(in[a]);
    }
    free(out); free(in); free(no); free(nin);
    *grp = rp2; *gci = ci2; *gS = f2;
}

/* Drop and rescale the entries of every row of P as for one interpolation row. */
static bsr* truncate_matrix(const bsr* P, double trunc, int pmax) {
    int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (P->nnzb > 0 ? P->nnzb : 1));
    double* w = (double*)malloc(sizeof(double) * (P->nnzb > 0 ? P->nnzb : 1));
    int64_t* cnt = (int64_t*)calloc(P->nr > 0 ? P->nr : 1, sizeof(int64_t));
    memcpy(col, P->ci, sizeof(int32_t) * P->nnzb);
    memcpy(w, P->v, sizeof(double) * P->nnzb);
    for (int64_t i = 0; i < P->nr; ++i)
        cnt[i] = truncate_row(col + P->rp[i], w + P->rp[i], P->rp[i + 1] - P->rp[i], trunc, pmax);
    int64_t nnz = 0;
    for (int64_t i = 0; i < P->nr; ++i) nnz += cnt[i];
    bsr* T = bsr_new(P->nr, P->nc, 1, 1, nnz);
    for (int64_t i = 0; i < P->nr; ++i) {
        T->rp[i + 1] = T->rp[i] + (int32_t)cnt[i];
        memcpy(T->ci + T->rp[i], col + P->rp[i], sizeof(int32_t) * cnt[i]);
        memcpy(T->v + T->rp[i], w + P->rp[i], sizeof(double) * cnt[i]);
    }
    free(col); free(w); free(cnt);
    return T;
}

/* One aggressive level: HMIS on S (first stage), HMIS on the second-stage graph of its C points,
 * P = truncation of P1 P2 with P1 = extended+i of A onto the first-stage C points and P2 =
 * extended+i of A1 = P1^T A P1 onto the second-stage C points.  Writes L->agg (coarse index of
 * the final C points, -1 elsewhere) and L->P; returns the number of coarse points, or -1. */
static int64_t aggressive_level(level* L, const amg_opts* o, int l) {
    const bsr* A = L->A;
    int64_t n = A->nr;
    int8_t* cf = (int8_t*)malloc(n > 0 ? n : 1);
    int8_t* first = (int8_t*)malloc(n > 0 ? n : 1);
    if (orc_cl_hmis(n, A->rp, A->ci, L->strong, o->hmis_domain, o->seed, l, cf, first)) { free(cf); free(first); return -1; }
    int32_t* c1 = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t n1 = 0;
    for (int64_t i = 0; i < n; ++i) c1[i] = cf[i] == 1 ? (int32_t)n1++ : -1;
    int32_t *grp, *gci;
    uint8_t* gS;
    second_stage_graph(n, A->rp, A->ci, L->strong, c1, n1, &grp, &gci, &gS);
    int8_t* cf2 = (int8_t*)malloc(n1 > 0 ? n1 : 1);
    int8_t* first2 = (int8_t*)malloc(n1 > 0 ? n1 : 1);
    int rc = orc_cl_hmis(n1, grp, gci, gS, o->hmis_domain, o->seed, l + 32, cf2, first2);
    free(grp); free(gci); free(gS); free(first2); free(cf); free(first);
    if (rc) { free(c1); free(cf2); return -1; }
    int32_t* c2 = (int32_t*)malloc(sizeof(int32_t) * (n1 > 0 ? n1 : 1));
    int64_t n2 = 0;
    for (int64_t a = 0; a < n1; ++a) c2[a] = cf2[a] == 1 ? (int32_t)n2++ : -1;
    free(cf2);
    L->agg = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) L->agg[i] = c1[i] >= 0 ? c2[c1[i]] : -1;
    if (n2 <= 0) { free(c1); free(c2); return n2; }
    bsr* P1 = extpi(n, n1, A->rp, A->ci, A->v, L->func, L->strong, c1, o->trunc, o->pmax);
    bsr* R1 = transpose(P1);
    bsr* AP1 = spgemm(A, P1);
    bsr* A1 = spgemm(R1, AP1);
    bsr_free(R1); bsr_free(AP1);
    uint8_t* f1 = (uint8_t*)malloc(n1 > 0 ? n1 : 1);
    for (int64_t i = 0; i < n; ++i)
        if (c1[i] >= 0) f1[c1[i]] = L->func[i];
    uint8_t* S1 = (uint8_t*)malloc(A1->nnzb > 0 ? A1->nnzb : 1);
    orc_cl_strength(n1, A1->rp, A1->ci, A1->v, f1, o->cl_theta, S1);
    bsr* P2 = extpi(n1, n2, A1->rp, A1->ci, A1->v, f1, S1, c2, o->trunc, o->pmax);
    bsr* P12 = spgemm(P1, P2);
    L->P = truncate_matrix(P12, o->trunc, o->pmax);
    bsr_free(P1); bsr_free(A1); bsr_free(P2); bsr_free(P12);
    free(S1); free(f1); free(c1); free(c2);
    return n2;
}

/* One standard level: HMIS on S and extended+i onto its C points.  Writes L->agg and L->P (P only
 * when there are C points); returns the number of coarse points, or -1. */
static int64_t standard_level(level* L, const amg_opts* o, int l) {
    const bsr* A = L->A;
    int64_t n = A->nr;
    int8_t* cf = (int8_t*)malloc(n > 0 ? n : 1);
    int8_t* first = (int8_t*)malloc(n > 0 ? n : 1);
    if (orc_cl_hmis(n, A->rp, A->ci, L->strong, o->hmis_domain, o->seed, l, cf, first)) { free(cf); free(first); return -1; }
    free(first);
    L->agg = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) L->agg[i] = cf[i] == 1 ? (int32_t)nc++ : -1;
    free(cf);
    if (nc > 0) L->P = extpi(n, nc, A->rp, A->ci, A->v, L->func, L->strong, L->agg, o->trunc, o->pmax);
    return nc;
}

/* test entry: the second-stage graph of a split (cf: 1 C, -1 F); grp (n1 + 1) always, gci/gS
 * (entries) when not NULL; returns the number of entries */
int64_t orc_cl_second_stage(int64_t n, const int32_t* rp, const int32_t* ci, const uint8_t* S, const int8_t* cf,
                            int32_t* grp, int32_t* gci, uint8_t* gS) {
    int32_t* c1 = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t n1 = 0;
    for (int64_t i = 0; i < n; ++i) c1[i] = cf[i] == 1 ? (int32_t)n1++ : -1;
    int32_t *r2, *c2;
    uint8_t* f2;
    second_stage_graph(n, rp, ci, S, c1, n1, &r2, &c2, &f2);
    memcpy(grp, r2, sizeof(int32_t) * (n1 + 1));
    if (gci) memcpy(gci, c2, sizeof(int32_t) * r2[n1]);
    if (gS) memcpy(gS, f2, r2[n1]);
    int64_t nnz = r2[n1];
    free(r2); free(c2); free(f2); free(c1);
    return nnz;
}

static amg* amg_build_classical(const bsr* A0, const amg_opts* o) {
    amg* h = (amg*)calloc(1, sizeof(amg));
    h->o = *o;
    level* L = &h->L[0];
    L->A = to_scalar(A0, &L->func);
    L->b = 1; L->k = 1;
    int l = 0;
    int64_t maxn = 0;
    for (;;) {
        L = &h->L[l];
        int64_t n = L->A->nr;
        if (n > maxn) maxn = n;
        if (n <= o->coarse_max || l + 1 >= o->max_levels || l + 1 >= MAXLEV) break;
        L->strong = (uint8_t*)malloc(L->A->nnzb > 0 ? L->A->nnzb : 1);
        orc_cl_strength(n, L->A->rp, L->A->ci, L->A->v, L->func, o->cl_theta, L->strong);
        int64_t nc = l < o->agg_levels ? aggressive_level(L, o, l) : standard_level(L, o, l);
        if (nc < 0) { orc_amg_free(h); return NULL; }
        if (nc == 0 || (double)nc > o->max_coarse_ratio * (double)n) {
            free(L->agg); L->agg = NULL; free(L->strong); L->strong = NULL;
            bsr_free(L->P); L->P = NULL;
            break;
        }
        L->n_agg = nc;
        L->R = transpose(L->P);
        bsr* AP = spgemm(L->A, L->P);
        level* N = &h->L[l + 1];
        N->A = spgemm(L->R, AP);
        bsr_free(AP);
        N->b = 1; N->k = 1;
        N->func = (uint8_t*)malloc(nc > 0 ? nc : 1);
        for (int64_t i = 0; i < n; ++i)
            if (L->agg[i] >= 0) N->func[L->agg[i]] = L->func[i];
        ++l;
    }
    h->nlev = l + 1;
    for (int t = 0; t + 1 < h->nlev; ++t) {
        if (level_diag(&h->L[t])) { orc_amg_free(h); return NULL; }
        if (o->l1_gs) {
            h->L[t].ell = (double*)malloc(sizeof(double) * (h->L[t].A->nr > 0 ? h->L[t].A->nr : 1));
            l1_diag(h->L[t].A, o->gs_domain, h->L[t].ell, h->L[t].Dinv);
        }
    }
    if (coarse_factor(h)) { orc_amg_free(h); return NULL; }
    h->work = (double*)malloc(sizeof(double) * 6 * (maxn + 8));
    return h;
}

/* Numeric re-setup (a reuse of the hierarchy when the matrix values change and its pattern does
 * not): level 0 takes the new values (and, if B0 is not NULL, a new near-null space); the
 * strength flags, MIS-2 roots and aggregates of every level are kept; every value-dependent
 * quantity is recomputed level by level exactly as in a full setup. */
static int amg_update(amg* h, const double* vals0, const double* B0) {
    level* L0 = &h->L[0];
    if (h->o.amg_type == 1) {
        /* classical: the splitting and the interpolation depend on the values; set up again */
        bsr A = *L0->A;
        A.v = (double*)vals0;
        amg* h2 = amg_build_classical(&A, &h->o);
        if (!h2) return -1;
        int64_t vc = h->vcycles;
        for (int l = 0; l < h->nlev; ++l) level_free(&h->L[l]);
        free(h->LU); free(h->piv); free(h->work);
        *h = *h2;
        h->vcycles = vc;
        free(h2);
        return 0;
    }
    memcpy(L0->A->v, vals0, sizeof(double) * L0->A->nnzb * L0->b * L0->b);
    if (B0) memcpy(L0->B, B0, sizeof(double) * L0->A->nr * L0->b * L0->k);
    for (int l = 0; l + 1 < h->nlev; ++l)
        if (level_numeric(h, l)) return -1;
    return coarse_factor(h);
}

int orc_amg_update(amg* h, const double* vals0, const double* B0) { return amg_update(h, vals0, B0); }

/* Build the hierarchy for the square b x b BSR matrix A0 with near-null space B0 ((nr*b) x k).
 * A0 is copied.  Returns NULL on failure. */
static amg* amg_build(const bsr* A0, const double* B0, int k, const amg_opts* o) {
    if (o->amg_type == 1) return amg_build_classical(A0, o);
    amg* h = (amg*)calloc(1, sizeof(amg));
    h->o = *o;
    level* L = &h->L[0];
    L->A = bsr_new(A0->nr, A0->nc, A0->br, A0->bc, A0->nnzb);
    memcpy(L->A->rp, A0->rp, sizeof(int32_t) * (A0->nr + 1));
    memcpy(L->A->ci, A0->ci, sizeof(int32_t) * A0->nnzb);
    memcpy(L->A->v, A0->v, sizeof(double) * A0->nnzb * A0->br * A0->bc);
    L->b = A0->br; L->k = k;
    L->B = (double*)malloc(sizeof(double) * A0->nr * A0->br * k);
    memcpy(L->B, B0, sizeof(double) * A0->nr * A0->br * k);
    int l = 0;
    int64_t maxn = 0;
    for (;;) {
        L = &h->L[l];
        int64_t n = L->A->nr * L->b;
        if (n > maxn) maxn = n;
        if (n <= o->coarse_max || l + 1 >= o->max_levels || l + 1 >= MAXLEV) break;
        int64_t nr = L->A->nr;
        L->strong = (uint8_t*)malloc(L->A->nnzb > 0 ? L->A->nnzb : 1);
        uint8_t* iso = (uint8_t*)malloc(nr);
        uint8_t* root = (uint8_t*)malloc(nr);
        double theta = ldexp(o->theta, -l);
        orc_strength(nr, L->b, L->A->rp, L->A->ci, L->A->v, theta, L->strong, iso);
        orc_mis2(nr, L->A->rp, L->A->ci, L->strong, iso, o->seed, l, root);
        L->agg = (int32_t*)malloc(sizeof(int32_t) * nr);
        L->n_agg = orc_aggregate(nr, L->A->rp, L->A->ci, L->strong, iso, root, o->seed, l, L->agg);
        free(iso); free(root);
        if (L->n_agg <= 0 || (double)(L->n_agg * L->k) > o->max_coarse_ratio * (double)n) {
            free(L->agg); L->agg = NULL; free(L->strong); L->strong = NULL; L->n_agg = 0;
            break;
        }
        if (level_numeric(h, l)) { orc_amg_free(h); return NULL; }
        ++l;
    }
    h->nlev = l + 1;
    /* smoother data on every level above the coarsest */
    for (int t = 0; t + 1 < h->nlev; ++t)
        if (!h->L[t].Dinv && level_diag(&h->L[t])) { orc_amg_free(h); return NULL; }
    if (coarse_factor(h)) { orc_amg_free(h); return NULL; }
    h->work = (double*)malloc(sizeof(double) * 6 * (maxn + 8));
    return h;
}

/* Smoother on level l: x <- x + smoothing steps for A x = b (x0 = x, or 0 if zero_init). */
static void smooth(const amg* h, int l, const double* b, double* x, int zero_init, double* r, double* d, double* z) {
    const level* L = &h->L[l];
    int64_t n = L->A->nr * L->b;
    int bs = L->b, bb = bs * bs;
    if (zero_init) memset(x, 0, sizeof(double) * n);
    #define DINV_APPLY(src, dst) do { \
        _Pragma("omp parallel for schedule(static) if (n > PAR_MIN)") \
        for (int64_t i_ = 0; i_ < L->A->nr; ++i_) \
            for (int r_ = 0; r_ < bs; ++r_) { double s_ = 0.0; \
                for (int c_ = 0; c_ < bs; ++c_) s_ += L->Dinv[i_ * bb + r_ * bs + c_] * (src)[i_ * bs + c_]; \
                (dst)[i_ * bs + r_] = s_; } } while (0)
    if (h->o.smoother == 0) {
        double w = 4.0 / (3.0 * L->lam);
        for (int s = 0; s < h->o.jacobi_sweeps; ++s) {
            bsr_mv(L->A, x, r);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
            DINV_APPLY(r, z);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t i = 0; i < n; ++i) x[i] += w * z[i];
        }
    } else {
        double lmax = L->lam, lmin = L->lam / h->o.cheb_ratio;
        double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
        double sigma = theta / delta, rho_prev = 1.0 / sigma;
        bsr_mv(L->A, x, r);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        DINV_APPLY(r, z);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
        for (int64_t i = 0; i < n; ++i) { d[i] = z[i] / theta; x[i] += d[i]; }
        for (int s = 1; s < h->o.cheb_degree; ++s) {
            bsr_mv(L->A, x, r);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
            DINV_APPLY(r, z);
            double rho = 1.0 / (2.0 * sigma - rho_prev);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t i = 0; i < n; ++i) { d[i] = rho * rho_prev * d[i] + (2.0 * rho / delta) * z[i]; x[i] += d[i]; }
            rho_prev = rho;
        }
    }
    #undef DINV_APPLY
}

static void vcycle_rec(amg* h, int l, const double* b, double* x) {
    level* L = &h->L[l];
    int64_t n = L->A->nr * L->b;
    if (l == h->nlev - 1) {
        memcpy(x, b, sizeof(double) * n);
        lu_solve(n, h->LU, h->piv, x);
        return;
    }
    double* r = (double*)malloc(sizeof(double) * n);
    double* d = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    if (h->o.amg_type == 1) hybrid_gs(L->A, L->Dinv, L->ell, h->o.gs_domain, 0, b, NULL, x);
    else smooth(h, l, b, x, 1, r, d, z);
    bsr_mv(L->A, x, r);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    int64_t nc = L->R->nr * L->R->br;
    double* bc = (double*)malloc(sizeof(double) * nc);
    double* xc = (double*)malloc(sizeof(double) * nc);
    bsr_mv(L->R, r, bc);
    vcycle_rec(h, l + 1, bc, xc);
    bsr_mv(L->P, xc, z);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
    for (int64_t i = 0; i < n; ++i) x[i] += z[i];
    if (h->o.amg_type == 1) {
        memcpy(d, x, sizeof(double) * n);
        hybrid_gs(L->A, L->Dinv, L->ell, h->o.gs_domain, 1, b, d, x);
    } else {
        smooth(h, l, b, x, 0, r, d, z);
    }
    free(r); free(d); free(z); free(bc); free(xc);
}

/* x = V-cycle(b) with zero initial guess */
void orc_amg_vcycle(amg* h, const double* b, double* x) {
    h->vcycles++;
    vcycle_rec(h, 0, b, x);
}

/* One application of the level-l smoother (tests). */
void orc_amg_smooth(amg* h, int l, const double* b, double* x, int zero_init) {
    int64_t n = h->L[l].A->nr * h->L[l].b;
    double* r = (double*)malloc(sizeof(double) * n);
    double* d = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    if (h->o.amg_type == 1) {
        /* classical: the V-cycle's sweeps (forward from zero, or backward from x) */
        if (zero_init) hybrid_gs(h->L[l].A, h->L[l].Dinv, h->L[l].ell, h->o.gs_domain, 0, b, NULL, x);
        else { memcpy(d, x, sizeof(double) * n); hybrid_gs(h->L[l].A, h->L[l].Dinv, h->L[l].ell, h->o.gs_domain, 1, b, d, x); }
    } else {
        smooth(h, l, b, x, zero_init, r, d, z);
    }
    free(r); free(d); free(z);
}

/* Generic entry: hierarchy for a square BSR (b x b blocks) with near-null space B. */
int orc_amg_create(int64_t nr, int b, const int32_t* rp, const int32_t* ci, const double* val,
                   const double* B, int k, const amg_opts* o, amg** out) {
    bsr A = {nr, nr, b, b, rp[nr], (int32_t*)rp, (int32_t*)ci, (double*)val};
    amg* h = amg_build(&A, B, k, o);
    *out = h;
    return h ? 0 : -1;
}

int orc_amg_nlevels(const amg* h) { return h->nlev; }

/* info: [nr, b, k, nnzb(A), n_agg, nnzb(P), nnzb(R), ncoarse] ; lam returned separately */
void orc_amg_level_info(const amg* h, int l, int64_t* info, double* lam) {
    const level* L = &h->L[l];
    info[0] = L->A->nr; info[1] = L->b; info[2] = L->k; info[3] = L->A->nnzb;
    info[4] = L->n_agg; info[5] = L->P ? L->P->nnzb : 0; info[6] = L->R ? L->R->nnzb : 0;
    info[7] = h->ncoarse;
    *lam = L->lam;
}

/* field: 0 A.rp 1 A.ci 2 A.v 3 agg (classical: coarse index or -1) 4 P.rp 5 P.ci 6 P.v 7 R.rp
 * 8 R.ci 9 R.v 10 strong 11 dead 12 Dinv 13 B 14 Q 15 func (classical) */
int orc_amg_level_get(const amg* h, int l, int field, void* dst) {
    const level* L = &h->L[l];
    const bsr* M = NULL;
    switch (field) {
        case 0: case 1: case 2: M = L->A; break;
        case 4: case 5: case 6: M = L->P; break;
        case 7: case 8: case 9: M = L->R; break;
    }
    if ((field <= 9 && field != 3) && !M) return -1;
    switch (field) {
        case 0: case 4: case 7: memcpy(dst, M->rp, sizeof(int32_t) * (M->nr + 1)); break;
        case 1: case 5: case 8: memcpy(dst, M->ci, sizeof(int32_t) * M->nnzb); break;
        case 2: case 6: case 9: memcpy(dst, M->v, sizeof(double) * M->nnzb * M->br * M->bc); break;
        case 3: if (!L->agg) return -1; memcpy(dst, L->agg, sizeof(int32_t) * L->A->nr); break;
        case 10: if (!L->strong) return -1; memcpy(dst, L->strong, L->A->nnzb); break;
        case 11: if (!L->dead) return -1; memcpy(dst, L->dead, L->n_agg * L->k); break;
        case 12: if (!L->Dinv) return -1; memcpy(dst, L->Dinv, sizeof(double) * L->A->nr * L->b * L->b); break;
        case 13: if (!L->B) return -1; memcpy(dst, L->B, sizeof(double) * L->A->nr * L->b * L->k); break;
        case 14: if (!L->Q) return -1; memcpy(dst, L->Q, sizeof(double) * L->A->nr * L->b * L->k); break;
        case 15: if (!L->func) return -1; memcpy(dst, L->func, L->A->nr); break;
        default: return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ Krylov */
typedef void (*op_fn)(void* ctx, const double* x, double* y);

/* sum_i a_i b_i: each chunk of DOT_CHUNK entries summed in order, then the chunk sums in order
 * (the same result on any number of threads) */
static double dot(int64_t n, const double* a, const double* b) {
    int64_t nch = (n + DOT_CHUNK - 1) / DOT_CHUNK;
    if (nch <= 1) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
        return s;
    }
    double* part = (double*)malloc(sizeof(double) * nch);
#pragma omp parallel for schedule(static) if (nch > 8)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t e = (c + 1) * DOT_CHUNK < n ? (c + 1) * DOT_CHUNK : n;
        double s = 0.0;
        for (int64_t i = c * DOT_CHUNK; i < e; ++i) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nch; ++c) s += part[c];
    free(part);
    return s;
}

typedef struct { int64_t iters; double rel_res; int converged; } kstat;

/* Right-preconditioned flexible GMRES(m) for op(x) = b with preconditioner prec.
 * Stops when the Givens residual estimate |g_{j+1}| <= tol*||b||; if check_true, the true
 * residual is recomputed and the method restarts while it is above tol*||b||. */
static kstat fgmres(int64_t n, op_fn op, void* oc, op_fn prec, void* pc, const double* b, double* x,
                    double tol, int maxit, int m, int use_x0, int check_true) {
    kstat st = {0, 0.0, 0};
    double bn = sqrt(dot(n, b, b));
    if (!use_x0) memset(x, 0, sizeof(double) * n);
    if (bn == 0.0) { memset(x, 0, sizeof(double) * n); st.converged = 1; return st; }
    double* V = (double*)malloc(sizeof(double) * n * (m + 1));
    double* Z = (double*)malloc(sizeof(double) * n * m);
    double* w = (double*)malloc(sizeof(double) * n);
    double* H = (double*)malloc(sizeof(double) * (m + 1) * m);
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* g = (double*)malloc(sizeof(double) * (m + 1));
    double* y = (double*)malloc(sizeof(double) * m);
    int first = 1;
    double est = INFINITY;
    for (;;) {
        /* r = b - op(x) */
        if (first && !use_x0) memcpy(V, b, sizeof(double) * n);
        else {
            op(oc, x, w);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t i = 0; i < n; ++i) V[i] = b[i] - w[i];
        }
        first = 0;
        double beta = sqrt(dot(n, V, V));
        st.rel_res = beta / bn;
        if (beta <= tol * bn) { st.converged = 1; break; }
        if (!check_true && est <= tol * bn) { st.converged = 1; break; }
        if (st.iters >= maxit) break;
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
        for (int64_t i = 0; i < n; ++i) V[i] /= beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int j = 0;
        for (; j < m;) {
            prec(pc, V + (int64_t)j * n, Z + (int64_t)j * n);
            op(oc, Z + (int64_t)j * n, w);
            for (int i = 0; i <= j; ++i) {
                double hij = dot(n, w, V + (int64_t)i * n);
                H[i * m + j] = hij;
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
                for (int64_t e = 0; e < n; ++e) w[e] -= hij * V[(int64_t)i * n + e];
            }
            double hn = sqrt(dot(n, w, w));
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double rr = sqrt(a * a + c * c);
            cs[j] = (rr == 0.0) ? 1.0 : a / rr;
            sn[j] = (rr == 0.0) ? 0.0 : c / rr;
            H[j * m + j] = rr;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            st.iters++;
            ++j;
            est = fabs(g[j]);
            if (hn == 0.0) break;           /* happy breakdown */
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t e = 0; e < n; ++e) V[(int64_t)j * n + e] = w[e] / hn;
            if (est <= tol * bn || st.iters >= maxit) break;
        }
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t < j; ++t) s -= H[i * m + t] * y[t];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < j; ++i)
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t e = 0; e < n; ++e) x[e] += y[i] * Z[(int64_t)i * n + e];
        st.rel_res = est / bn;
        if (!check_true && (est <= tol * bn || st.iters >= maxit)) { st.converged = est <= tol * bn; break; }
    }
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y);
    return st;
}

/* PCG (flexible = 0) or flexible CG with the Polak-Ribiere beta of Notay (flexible = 1). */
static kstat pcg(int64_t n, op_fn op, void* oc, op_fn prec, void* pc, const double* b, double* x,
                 double tol, int maxit, int flexible) {
    kstat st = {0, 0.0, 0};
    double bn = sqrt(dot(n, b, b));
    memset(x, 0, sizeof(double) * n);
    if (bn == 0.0) { st.converged = 1; return st; }
    double* r = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    double* rold = (double*)malloc(sizeof(double) * n);
    memcpy(r, b, sizeof(double) * n);
    prec(pc, r, z);
    memcpy(p, z, sizeof(double) * n);
    double rz = dot(n, r, z);
    for (;;) {
        op(oc, p, q);
        double alpha = rz / dot(n, p, q);
        memcpy(rold, r, sizeof(double) * n);
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        st.iters++;
        double rn = sqrt(dot(n, r, r));
        st.rel_res = rn / bn;
        if (rn <= tol * bn) { st.converged = 1; break; }
        if (st.iters >= maxit) break;
        prec(pc, r, z);
        double rz_new = dot(n, r, z);
        double beta;
        if (flexible) {
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
            for (int64_t i = 0; i < n; ++i) rold[i] = r[i] - rold[i];
            beta = dot(n, z, rold) / rz;        /* z . (r_new - r_old) */
        } else beta = rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static) if (n > PAR_MIN)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    free(r); free(z); free(p); free(q); free(rold);
    return st;
}

/* ------------------------------------------------------------------ SCR */
typedef struct {
    double tol, tol_A, tol_S, tol_I;
    int max_it, max_it_A, max_it_S, max_it_I;
    int restart, restart_inner;
    int use_x0;
    int flexible_cg;
    int precond;         /* 0 SCR (Algorithm 1), 1 SIMPLE-type block preconditioner (Sec. 5.2.1) */
} solve_opts;

typedef struct {
    int outer_it;
    double rel_res_true;
    int64_t calls_A, its_A, calls_S, its_S, calls_I, its_I, vcycles_A, vcycles_S;
    int converged;
} scr_stats;

typedef struct {
    int64_t nb;
    bsr *K, *A, *G, *D, *C, *Sh;
    double* diagA;
    amg *amgA, *amgS;
    int schur_diag;
    solve_opts so;
    scr_stats st;
    double *t1, *t2, *t3;   /* scratch */
    /* outlet resistance coupling: outlet k adds m_k a_k a_k^T to the velocity block; its entries
     * out_off[k] .. out_off[k+1]-1 name a block row and the 3 velocity components of a_k there */
    int n_out;
    int64_t* out_off; int32_t* out_blk; double *out_a, *out_m;
} scr;

/* yv += sum_k m_k a_k (a_k . xv) on velocity vectors (3 per block row), outlets in order, each
 * dot product summed over its entries in order (Sec. 3.5, the linearised reduced outlet models) */
static void add_outlets(const scr* s, const double* xv, double* yv) {
    for (int k = 0; k < s->n_out; ++k) {
        double dot = 0.0;
        for (int64_t e = s->out_off[k]; e < s->out_off[k + 1]; ++e)
            for (int i = 0; i < 3; ++i) dot += s->out_a[3 * e + i] * xv[3 * (int64_t)s->out_blk[e] + i];
        double c = s->out_m[k] * dot;
        for (int64_t e = s->out_off[k]; e < s->out_off[k + 1]; ++e)
            for (int i = 0; i < 3; ++i) yv[3 * (int64_t)s->out_blk[e] + i] += c * s->out_a[3 * e + i];
    }
}

static void op_K(void* c, const double* x, double* y) {
    /* split layout: x = [x_v (3nb); x_p (nb)] */
    scr* s = (scr*)c;
    int64_t nb = s->nb;
#pragma omp parallel for schedule(static) if (nb > PAR_MIN)
    for (int64_t i = 0; i < nb; ++i) {
        double acc[4] = {0};
        for (int32_t q = s->K->rp[i]; q < s->K->rp[i + 1]; ++q) {
            int32_t j = s->K->ci[q];
            const double* blk = s->K->v + (int64_t)q * 16;
            double xj[4] = {x[3 * j], x[3 * j + 1], x[3 * j + 2], x[3 * nb + j]};
            for (int r = 0; r < 4; ++r)
                for (int cc = 0; cc < 4; ++cc) acc[r] += blk[4 * r + cc] * xj[cc];
        }
        y[3 * i] = acc[0]; y[3 * i + 1] = acc[1]; y[3 * i + 2] = acc[2]; y[3 * nb + i] = acc[3];
    }
    add_outlets(s, x, y);
}
static void op_A(void* c, const double* x, double* y) {
    bsr_mv(((scr*)c)->A, x, y);
    add_outlets((scr*)c, x, y);
}
static void prec_A(void* c, const double* x, double* y) { scr* s = (scr*)c; s->st.vcycles_A++; orc_amg_vcycle(s->amgA, x, y); }
static void prec_S(void* c, const double* x, double* y) { scr* s = (scr*)c; s->st.vcycles_S++; orc_amg_vcycle(s->amgS, x, y); }

/* Algorithm 2: S x_p = C x_p - D (A^-1 (G x_p)), A^-1 by GMRES+AMG(A) to tol_I */
static void op_S(void* c, const double* xp, double* y) {
    scr* s = (scr*)c;
    int64_t nb = s->nb;
    double* xbar = (double*)malloc(sizeof(double) * 3 * nb);
    double* xt = (double*)malloc(sizeof(double) * 3 * nb);
    double* t = (double*)malloc(sizeof(double) * nb);
    bsr_mv(s->G, xp, xbar);
    kstat k = fgmres(3 * nb, op_A, s, prec_A, s, xbar, xt, s->so.tol_I, s->so.max_it_I, s->so.restart_inner, 0, 0);
    s->st.calls_I++; s->st.its_I += k.iters;
    bsr_mv(s->D, xt, t);
    bsr_mv(s->C, xp, y);
    for (int64_t i = 0; i < nb; ++i) y[i] -= t[i];
    free(xbar); free(xt); free(t);
}

/* Algorithm 1 (with step 2 read as r_p <- r_p - D y^_v):  y = P_SCR^-1 r */
static void prec_SCR(void* c, const double* r, double* y) {
    scr* s = (scr*)c;
    int64_t nb = s->nb;
    const double* rv = r;
    const double* rp = r + 3 * nb;
    double* yv = y;
    double* yp = y + 3 * nb;
    double* yhat = (double*)malloc(sizeof(double) * 3 * nb);
    double* tp = (double*)malloc(sizeof(double) * nb);
    double* tv = (double*)malloc(sizeof(double) * 3 * nb);
    kstat k = fgmres(3 * nb, op_A, s, prec_A, s, rv, yhat, s->so.tol_A, s->so.max_it_A, s->so.restart_inner, 0, 0);
    s->st.calls_A++; s->st.its_A += k.iters;
    bsr_mv(s->D, yhat, tp);
    for (int64_t i = 0; i < nb; ++i) tp[i] = rp[i] - tp[i];
    k = fgmres(nb, op_S, s, prec_S, s, tp, yp, s->so.tol_S, s->so.max_it_S, s->so.restart_inner, 0, 0);
    s->st.calls_S++; s->st.its_S += k.iters;
    bsr_mv(s->G, yp, tv);
    for (int64_t i = 0; i < 3 * nb; ++i) tv[i] = rv[i] - tv[i];
    k = fgmres(3 * nb, op_A, s, prec_A, s, tv, yv, s->so.tol_A, s->so.max_it_A, s->so.restart_inner, 0, 0);
    s->st.calls_A++; s->st.its_A += k.iters;
    free(yhat); free(tp); free(tv);
}

/* SIMPLE (Sec. 5.2.1): the inverse of the product P = [I 0; D A^-1 I] [A 0; 0 S^] [I d^-1 G; 0 I]
 * applied to r, with A^-1 by GMRES+AMG(A) to tol_A and S^^-1 by GMRES+AMG(S^) on the explicit
 * sparse S^ to tol_S (no inner-level solver):
 *   y*_v = A^-1 r_v;  y_p = S^^-1 (r_p - D y*_v);  y_v = y*_v - d^-1 (G y_p).
 * d is the diagonal of A (SIMPLE) or its absolute row sums (SIMPLEC), the same d as in S^. */
static void op_Sh(void* c, const double* x, double* y) { bsr_mv(((scr*)c)->Sh, x, y); }
static void prec_SIMPLE(void* c, const double* r, double* y) {
    scr* s = (scr*)c;
    int64_t nb = s->nb;
    const double* rv = r;
    const double* rp = r + 3 * nb;
    double* yv = y;
    double* yp = y + 3 * nb;
    double* ystar = (double*)malloc(sizeof(double) * 3 * nb);
    double* tp = (double*)malloc(sizeof(double) * nb);
    double* tv = (double*)malloc(sizeof(double) * 3 * nb);
    kstat k = fgmres(3 * nb, op_A, s, prec_A, s, rv, ystar, s->so.tol_A, s->so.max_it_A, s->so.restart_inner, 0, 0);
    s->st.calls_A++; s->st.its_A += k.iters;
    bsr_mv(s->D, ystar, tp);
    for (int64_t i = 0; i < nb; ++i) tp[i] = rp[i] - tp[i];
    k = fgmres(nb, op_Sh, s, prec_S, s, tp, yp, s->so.tol_S, s->so.max_it_S, s->so.restart_inner, 0, 0);
    s->st.calls_S++; s->st.its_S += k.iters;
    bsr_mv(s->G, yp, tv);
    for (int64_t i = 0; i < 3 * nb; ++i) yv[i] = ystar[i] - tv[i] / s->diagA[i];
    free(ystar); free(tp); free(tv);
}

/* Split K (4x4 BSR) into A (3x3), G (3x1), D (1x3), C (1x1), all on K's block pattern. */
static void split_blocks(const bsr* K, bsr** A, bsr** G, bsr** D, bsr** Cm) {
    int64_t nb = K->nr, nz = K->nnzb;
    *A = bsr_new(nb, nb, 3, 3, nz); *G = bsr_new(nb, nb, 3, 1, nz);
    *D = bsr_new(nb, nb, 1, 3, nz); *Cm = bsr_new(nb, nb, 1, 1, nz);
    bsr* all[4] = {*A, *G, *D, *Cm};
    for (int t = 0; t < 4; ++t) {
        memcpy(all[t]->rp, K->rp, sizeof(int32_t) * (nb + 1));
        memcpy(all[t]->ci, K->ci, sizeof(int32_t) * nz);
    }
    for (int64_t q = 0; q < nz; ++q) {
        const double* k = K->v + q * 16;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) (*A)->v[q * 9 + 3 * i + j] = k[4 * i + j];
            (*G)->v[q * 3 + i] = k[4 * i + 3];
            (*D)->v[q * 3 + i] = k[12 + i];
        }
        (*Cm)->v[q] = k[15];
    }
}

/* S^ = C - D d^-1 G on the union of the patterns of C and D*G (structural), with d (one entry per
 * velocity dof) the diagonal of A (mode 0) or the sums of the absolute values of its rows (mode 1,
 * the SIMPLEC lumping). */
static bsr* schur_approx(const bsr* A, const bsr* G, const bsr* D, const bsr* Cm, double* diagA, int mode) {
    int64_t nb = A->nr;
    for (int64_t i = 0; i < nb; ++i) {
        if (mode == 0) {
            int32_t q = find_in_row(A, i, (int32_t)i);
            for (int c = 0; c < 3; ++c) diagA[3 * i + c] = A->v[(int64_t)q * 9 + 4 * c];
        } else {
            for (int c = 0; c < 3; ++c) {
                double sum = 0.0;
                for (int32_t q = A->rp[i]; q < A->rp[i + 1]; ++q)
                    for (int k = 0; k < 3; ++k) sum += fabs(A->v[(int64_t)q * 9 + 3 * c + k]);
                diagA[3 * i + c] = sum;
            }
        }
    }
    bsr* X = bsr_new(nb, nb, 1, 3, D->nnzb);
    memcpy(X->rp, D->rp, sizeof(int32_t) * (nb + 1));
    memcpy(X->ci, D->ci, sizeof(int32_t) * D->nnzb);
    for (int64_t q = 0; q < D->nnzb; ++q)
        for (int c = 0; c < 3; ++c) X->v[q * 3 + c] = D->v[q * 3 + c] / diagA[3 * (int64_t)D->ci[q] + c];
    bsr* DG = spgemm(X, G);
    bsr_free(X);
    /* union with C */
    int32_t* rp = (int32_t*)calloc(nb + 1, sizeof(int32_t));
    int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * (DG->nnzb + Cm->nnzb));
    double* v = (double*)malloc(sizeof(double) * (DG->nnzb + Cm->nnzb));
    int64_t nz = 0;
    for (int64_t i = 0; i < nb; ++i) {
        int32_t a = DG->rp[i], ae = DG->rp[i + 1], c = Cm->rp[i], ce = Cm->rp[i + 1];
        while (a < ae || c < ce) {
            int32_t ca = a < ae ? DG->ci[a] : INT32_MAX, cc = c < ce ? Cm->ci[c] : INT32_MAX;
            if (ca == cc) { ci[nz] = ca; v[nz] = Cm->v[c] - DG->v[a]; ++a; ++c; }
            else if (ca < cc) { ci[nz] = ca; v[nz] = -DG->v[a]; ++a; }
            else { ci[nz] = cc; v[nz] = Cm->v[c]; ++c; }
            ++nz;
        }
        rp[i + 1] = (int32_t)nz;
    }
    bsr* S = bsr_new(nb, nb, 1, 1, nz);
    memcpy(S->rp, rp, sizeof(int32_t) * (nb + 1));
    memcpy(S->ci, ci, sizeof(int32_t) * nz);
    memcpy(S->v, v, sizeof(double) * nz);
    free(rp); free(ci); free(v); bsr_free(DG);
    return S;
}

/* Rigid-body modes of the velocity dofs (6 columns), coordinates shifted by their mean. */
static void rigid_modes(int64_t nb, const double* xyz, double* B) {
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int64_t i = 0; i < nb; ++i) { cx += xyz[3 * i]; cy += xyz[3 * i + 1]; cz += xyz[3 * i + 2]; }
    cx /= (double)nb; cy /= (double)nb; cz /= (double)nb;
    memset(B, 0, sizeof(double) * nb * 18);
    for (int64_t i = 0; i < nb; ++i) {
        double x = xyz[3 * i] - cx, y = xyz[3 * i + 1] - cy, z = xyz[3 * i + 2] - cz;
        double* r0 = B + (3 * i) * 6; double* r1 = r0 + 6; double* r2 = r1 + 6;
        r0[0] = 1.0; r1[1] = 1.0; r2[2] = 1.0;
        r0[3] = -y; r1[3] = x;
        r1[4] = -z; r2[4] = y;
        r0[5] = z;  r2[5] = -x;
    }
}

int orc_scr_create(int64_t nb, const int32_t* rp, const int32_t* ci, const double* val, const double* xyz,
                   const amg_opts* ao, scr** out) {
    scr* s = (scr*)calloc(1, sizeof(scr));
    s->nb = nb;
    s->K = bsr_new(nb, nb, 4, 4, rp[nb]);
    memcpy(s->K->rp, rp, sizeof(int32_t) * (nb + 1));
    memcpy(s->K->ci, ci, sizeof(int32_t) * rp[nb]);
    memcpy(s->K->v, val, sizeof(double) * rp[nb] * 16);
    split_blocks(s->K, &s->A, &s->G, &s->D, &s->C);
    s->diagA = (double*)malloc(sizeof(double) * 3 * nb);
    s->schur_diag = ao->schur_diag;
    s->Sh = schur_approx(s->A, s->G, s->D, s->C, s->diagA, ao->schur_diag);
    double* B = (double*)malloc(sizeof(double) * nb * 18);
    rigid_modes(nb, xyz, B);
    s->amgA = amg_build(s->A, B, 6, ao);
    free(B);
    double* ones = (double*)malloc(sizeof(double) * nb);
    for (int64_t i = 0; i < nb; ++i) ones[i] = 1.0;
    amg_opts oS = *ao;
    int sdeg = ao->schur_cheb_degree;
    if (sdeg < 0) sdeg = nb <= 1000000 ? 8 : (nb <= 3000000 ? 12 : 16);
    if (sdeg > 0) oS.cheb_degree = sdeg;
    if (ao->schur_cheb_ratio > 0) oS.cheb_ratio = ao->schur_cheb_ratio;
    s->amgS = amg_build(s->Sh, ones, 1, &oS);
    free(ones);
    *out = s;
    if (!s->amgA || !s->amgS) return -1;
    return 0;
}

/* Numeric re-setup for a new matrix with the same pattern (and, if xyz is not NULL, new node
 * coordinates): the split, d and S^ are recomputed (S^ keeps its structural pattern), and both
 * hierarchies are updated with their aggregates kept (amg_update). */
int orc_scr_update(scr* s, const double* val, const double* xyz) {
    int64_t nb = s->nb;
    memcpy(s->K->v, val, sizeof(double) * s->K->nnzb * 16);
    bsr_free(s->A); bsr_free(s->G); bsr_free(s->D); bsr_free(s->C); bsr_free(s->Sh);
    split_blocks(s->K, &s->A, &s->G, &s->D, &s->C);
    s->Sh = schur_approx(s->A, s->G, s->D, s->C, s->diagA, s->schur_diag);
    double* B = NULL;
    if (xyz) {
        B = (double*)malloc(sizeof(double) * nb * 18);
        rigid_modes(nb, xyz, B);
    }
    int rc = amg_update(s->amgA, s->A->v, B);
    free(B);
    if (rc) return -1;
    if (s->amgS->L[0].A->nnzb != s->Sh->nnzb) return -2;
    return amg_update(s->amgS, s->Sh->v, NULL);
}

/* Attach the outlet coupling (copied; n = 0 removes it).  The operators K and A of the solves
 * include it; the split, S^ and both hierarchies are those of the sparse K (they are not rebuilt). */
int orc_scr_set_outlets(scr* s, int n, const int64_t* off, const int32_t* blk, const double* a, const double* m) {
    free(s->out_off); free(s->out_blk); free(s->out_a); free(s->out_m);
    s->out_off = NULL; s->out_blk = NULL; s->out_a = NULL; s->out_m = NULL;
    s->n_out = 0;
    if (n <= 0) return 0;
    int64_t ne = off[n];
    for (int k = 0; k < n; ++k) if (off[k + 1] < off[k]) return -1;
    for (int64_t e = 0; e < ne; ++e) if (blk[e] < 0 || blk[e] >= s->nb) return -1;
    s->out_off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    s->out_blk = (int32_t*)malloc(sizeof(int32_t) * (ne > 0 ? ne : 1));
    s->out_a = (double*)malloc(sizeof(double) * 3 * (ne > 0 ? ne : 1));
    s->out_m = (double*)malloc(sizeof(double) * n);
    memcpy(s->out_off, off, sizeof(int64_t) * (n + 1));
    if (ne) { memcpy(s->out_blk, blk, sizeof(int32_t) * ne); memcpy(s->out_a, a, sizeof(double) * 3 * ne); }
    memcpy(s->out_m, m, sizeof(double) * n);
    s->n_out = n;
    return 0;
}

void orc_scr_free(scr* s) {
    if (!s) return;
    free(s->out_off); free(s->out_blk); free(s->out_a); free(s->out_m);
    bsr_free(s->K); bsr_free(s->A); bsr_free(s->G); bsr_free(s->D); bsr_free(s->C); bsr_free(s->Sh);
    free(s->diagA); orc_amg_free(s->amgA); orc_amg_free(s->amgS);
    free(s);
}

amg* orc_scr_amg(scr* s, int which) { return which == 0 ? s->amgA : s->amgS; }

/* Copy a split matrix: which 0 A, 1 G, 2 D, 3 C, 4 S^;  field 0 rp, 1 ci, 2 values.
 * info (if field < 0): [nr, nnzb, br, bc]. */
int orc_scr_matrix(const scr* s, int which, int field, void* dst) {
    const bsr* M = which == 0 ? s->A : which == 1 ? s->G : which == 2 ? s->D : which == 3 ? s->C : s->Sh;
    if (field < 0) { int64_t* info = (int64_t*)dst; info[0] = M->nr; info[1] = M->nnzb; info[2] = M->br; info[3] = M->bc; return 0; }
    if (field == 0) memcpy(dst, M->rp, sizeof(int32_t) * (M->nr + 1));
    else if (field == 1) memcpy(dst, M->ci, sizeof(int32_t) * M->nnzb);
    else memcpy(dst, M->v, sizeof(double) * M->nnzb * M->br * M->bc);
    return 0;
}

/* Interleaved [vx vy vz p] per node  <->  split [v (3nb); p (nb)] */
static void to_split(int64_t nb, const double* a, double* s) {
    for (int64_t i = 0; i < nb; ++i) {
        for (int c = 0; c < 3; ++c) s[3 * i + c] = a[4 * i + c];
        s[3 * nb + i] = a[4 * i + 3];
    }
}
static void from_split(int64_t nb, const double* s, double* a) {
    for (int64_t i = 0; i < nb; ++i) {
        for (int c = 0; c < 3; ++c) a[4 * i + c] = s[3 * i + c];
        a[4 * i + 3] = s[3 * nb + i];
    }
}

/* FGMRES(P_SCR) on K x = b; b and x interleaved (4 per node). */
int orc_scr_solve(scr* s, const double* b, double* x, const solve_opts* so, scr_stats* st) {
    int64_t nb = s->nb, n = 4 * nb;
    s->so = *so;
    memset(&s->st, 0, sizeof(s->st));
    double* bs = (double*)malloc(sizeof(double) * n);
    double* xs = (double*)malloc(sizeof(double) * n);
    to_split(nb, b, bs);
    if (so->use_x0) to_split(nb, x, xs);
    kstat k = fgmres(n, op_K, s, so->precond == 1 ? prec_SIMPLE : prec_SCR, s, bs, xs, so->tol, so->max_it,
                     so->restart, so->use_x0, 1);
    from_split(nb, xs, x);
    s->st.outer_it = (int)k.iters;
    s->st.rel_res_true = k.rel_res;
    s->st.converged = k.converged;
    s->st.vcycles_A = s->amgA->vcycles; s->st.vcycles_S = s->amgS->vcycles;
    if (st) *st = s->st;
    free(bs); free(xs);
    return k.converged ? 0 : 1;
}

/* Component operators on split vectors (tests):
 * op 0: y = K x (split 4nb)   1: y = A x (3nb)   2: y = V-cycle_A(x)   3: y = V-cycle_S^(x)
 *    4: y = S x by Algorithm 2 (nb)   5: y = P_SCR^-1 x by Algorithm 1 (split 4nb)
 *    6: y = G x (nb -> 3nb)   7: y = D x (3nb -> nb)   8: y = C x   9: y = S^ x
 *   10: y = P_SIMPLE^-1 x (split 4nb)   11: y = d, the diagonal used in S^ (3nb; x unused) */
int orc_scr_apply(scr* s, int op, const double* x, double* y, const solve_opts* so) {
    if (so) s->so = *so;
    switch (op) {
        case 0: op_K(s, x, y); break;
        case 1: op_A(s, x, y); break;
        case 2: orc_amg_vcycle(s->amgA, x, y); break;
        case 3: orc_amg_vcycle(s->amgS, x, y); break;
        case 4: op_S(s, x, y); break;
        case 5: prec_SCR(s, x, y); break;
        case 6: bsr_mv(s->G, x, y); break;
        case 7: bsr_mv(s->D, x, y); break;
        case 8: bsr_mv(s->C, x, y); break;
        case 9: bsr_mv(s->Sh, x, y); break;
        case 10: prec_SIMPLE(s, x, y); break;
        case 11: memcpy(y, s->diagA, sizeof(double) * 3 * s->nb); break;
        default: return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ mesh motion */
typedef struct { bsr* L; amg* h; int64_t n; } mesh;

static void op_L(void* c, const double* x, double* y) { bsr_mv(((mesh*)c)->L, x, y); }
static void prec_L(void* c, const double* x, double* y) { orc_amg_vcycle(((mesh*)c)->h, x, y); }

int orc_mesh_create(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const amg_opts* ao, mesh** out) {
    mesh* m = (mesh*)calloc(1, sizeof(mesh));
    m->n = n;
    m->L = bsr_new(n, n, 1, 1, rp[n]);
    memcpy(m->L->rp, rp, sizeof(int32_t) * (n + 1));
    memcpy(m->L->ci, ci, sizeof(int32_t) * rp[n]);
    memcpy(m->L->v, val, sizeof(double) * rp[n]);
    double* ones = (double*)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) ones[i] = 1.0;
    m->h = amg_build(m->L, ones, 1, ao);
    free(ones);
    *out = m;
    return m->h ? 0 : -1;
}
void orc_mesh_free(mesh* m) { if (!m) return; bsr_free(m->L); orc_amg_free(m->h); free(m); }
/* Numeric re-setup of the mesh hierarchy for new Laplacian values on the same pattern. */
int orc_mesh_update(mesh* m, const double* val) {
    memcpy(m->L->v, val, sizeof(double) * m->L->nnzb);
    return amg_update(m->h, val, NULL);
}
amg* orc_mesh_amg(mesh* m) { return m->h; }

/* Three independent CG solves (x, y, z components), b and x interleaved n x 3.
 * its[3] and rel[3] receive per-component iteration counts and final relative residuals. */
int orc_mesh_solve(mesh* m, const double* b, double* x, double tol, int maxit, int flexible, int64_t* its, double* rel) {
    int64_t n = m->n;
    double* bc = (double*)malloc(sizeof(double) * n);
    double* xc = (double*)malloc(sizeof(double) * n);
    int ok = 1;
    for (int c = 0; c < 3; ++c) {
        for (int64_t i = 0; i < n; ++i) bc[i] = b[3 * i + c];
        kstat k = pcg(n, op_L, m, prec_L, m, bc, xc, tol, maxit, flexible);
        for (int64_t i = 0; i < n; ++i) x[3 * i + c] = xc[i];
        its[c] = k.iters; rel[c] = k.rel_res;
        ok &= k.converged;
    }
    free(bc); free(xc);
    return ok ? 0 : 1;
}

/* Plain GMRES / FGMRES on a generic BSR with no preconditioner or with AMG (tests). */
typedef struct { bsr* M; amg* h; } gen_ctx;
static void op_gen(void* c, const double* x, double* y) { bsr_mv(((gen_ctx*)c)->M, x, y); }
static void prec_gen(void* c, const double* x, double* y) {
    gen_ctx* g = (gen_ctx*)c;
    if (g->h) orc_amg_vcycle(g->h, x, y);
    else memcpy(y, x, sizeof(double) * g->M->nr * g->M->br);
}
int orc_gmres(int64_t nr, int b, const int32_t* rp, const int32_t* ci, const double* val, amg* h,
              const double* rhs, double* x, double tol, int maxit, int restart, int64_t* its, double* rel) {
    bsr M = {nr, nr, b, b, rp[nr], (int32_t*)rp, (int32_t*)ci, (double*)val};
    gen_ctx g = {&M, h};
    kstat k = fgmres(nr * b, op_gen, &g, prec_gen, &g, rhs, x, tol, maxit, restart, 0, 1);
    *its = k.iters; *rel = k.rel_res;
    return k.converged ? 0 : 1;
}
int orc_cg(int64_t nr, const int32_t* rp, const int32_t* ci, const double* val, amg* h,
           const double* rhs, double* x, double tol, int maxit, int flexible, int64_t* its, double* rel) {
    bsr M = {nr, nr, 1, 1, rp[nr], (int32_t*)rp, (int32_t*)ci, (double*)val};
    gen_ctx g = {&M, h};
    kstat k = pcg(nr, op_gen, &g, prec_gen, &g, rhs, x, tol, maxit, flexible);
    *its = k.iters; *rel = k.rel_res;
    return k.converged ? 0 : 1;
}
