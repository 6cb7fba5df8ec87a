/*
 * synth.c -- seeded synthetic inputs for the SCR+AMG solver.
 *
 * This module builds the linear systems that the solver and the oracle are both given:
 * it holds the mesh, the P1 element integrals of the linearised unified-continuum VMS
 * tangent, the mesh-motion Laplacian and the right-hand sides.  It holds none of the
 * solver's arithmetic (no Krylov, no AMG, no Schur complement).
 *
 * Geometry.  A structured (i,j,k) index grid; the cross-section is mapped square->disk
 * shell by shell (shell s = max(|i-c|,|j-c|) goes to a circle of radius r_s), so the
 * lumen/wall interface is exactly the shell at r = R.  Each hexahedral cell is cut into
 * the six Kuhn tetrahedra along its diagonal; in the tube the index directions are
 * mirrored per quadrant so that the cut diagonal always points away from the axis
 * (conforming, and no cap-shaped slivers at the shell corners).
 *
 * Physics of the entries (fully discrete tangent of the paper's Section 3, divided by
 * alpha_f*gamma*dt; at rest every convective term vanishes, see the advective state below):
 *   fluid (Sec. 3.2, VMS):  A = rho*c_t*M (x) I3 + mu*Dev + tau_C*graddiv,
 *                           G = -(V/4) dN_a/dx_i,  D = -G^T,  C = tau_M * stiffness
 *   solid (Sec. 3.1 with c_m = c_c = 0, Sec. 3.5 tangent):
 *                           A = rho_s*c_t*M (x) I3 + (alpha_f*gamma*dt/alpha_m)*mu_s*Dev,
 *                           G, D as fluid,  C = (c_t/kappa) * M
 *   c_t = alpha_m/(alpha_f*gamma*dt); first-order generalized-alpha constants (Sec. 3.4).
 *   tau_M, tau_C from the element metric G = J^-T M J^-1 with the regular-simplex matrix M
 *   (Sec. 3.2, definition of the stabilisation parameters; the double sum over k,l).
 * Advective state (u_max != 0; tube and box only): the fluid nodes carry the Poiseuille profile
 * u = u_max (1 - r^2/R^2) e_z (r from the axis; box: R = half the narrower side, profile clipped
 * at zero).  It is a steady solution with zero fine-scale residual, so the VMS terms that carry
 * the state's v' or p' vanish, and the Oseen (frozen advection) tangent of Sec. 3.2 adds, per
 * fluid element with centroid velocity ub and constant grad u:
 *   A += rho N_a (ub.grad N_b) I + rho M_ab grad u                  (Galerkin convection, reaction)
 *      + tau_M rho^2 (ub.grad N_a) (c_t N_b + ub.grad N_b) I        (fine-scale momentum, SUPG form)
 *   G += tau_M rho (ub.grad N_a) dN_b/dx_i                          (v' through grad p)
 *   D += tau_M rho dN_a/dx_j (ub.grad N_b)                          (continuity, v' through (grad v) u)
 * with tau_M including ub.G.ub; element integrals by the centroid rule (exact for the mass-like
 * and gradient-gradient parts).  A is then nonsymmetric.
 * Outlets (tube and box): the outlet face z = z_max; per face triangle of a fluid element the
 * vector a of the resistance coupling (Sec. 3.5: a_Ai = integral of N_A n_i over the outlet)
 * gets area/3 * n at each vertex (n = +e_z); Dirichlet velocity dofs are zeroed.
 * Interface pressure duplication (Sec. 3.3): every node on the lumen/wall interface gets a
 * "virtual" block row right after it; solid elements use it for pressure, the physical
 * node for velocity; its velocity slots are identity rows.
 * Y-bifurcation (mode 2).  A uniform voxel grid of spacing h; the lumen is a union of three
 * branches (parent of radius R along +z ending at the junction, two daughters of radius rd*R
 * leaving the junction at angles th1, th2 from the z axis in the x-z plane), each a cylinder
 * with a spherical cap at the junction end and a flat cut at its free end; the wall is every
 * branch dilated to wall_ratio times its radius.  A voxel is kept when its centre lies in the
 * wall region; each kept voxel is cut into the six Kuhn tetrahedra (unmirrored), and a tetrahedron
 * is fluid when its centroid lies in the lumen.  The fluid/solid interface is the set of faces
 * between fluid and solid tetrahedra (a staircase, conforming by construction).  Velocity
 * Dirichlet: every node of the inlet plane, and solid-touching nodes within h of a daughter's
 * outlet cut; mesh motion Dirichlet: every node touching a solid tetrahedron, the inlet plane and
 * the outlet layers.
 * Mesh motion (Sec. 2.2.2 harmonic extension, stiffened by 1/element volume): scalar
 * Laplacian over all physical nodes; every node not strictly inside the lumen is Dirichlet.
 * Dirichlet dofs are eliminated symmetrically (row and column zeroed, unit diagonal).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int mode;        /* 0 = tube (disk-mapped shells), 1 = box (uniform, unmirrored Kuhn), 2 = Y voxels */
    int m_core;      /* tube: uniform core shells;          box: nx */
    int n_bl;        /* tube: boundary-layer shells;         box: ny */
    int n_wall;      /* tube: solid wall shells (0 = fluid only) */
    int nz;          /* cells along the axis */
    double R;        /* lumen radius;                        box: spacing h */
    double L;        /* length;                              box: unused (h used) */
    double wall_ratio; /* outer wall radius / R */
    double bl_ratio;   /* boundary-layer gradation factor */
    double rho_f, mu_f, rho_s, E_s, nu_s, dt, rho_inf;
    int terms;       /* bitmask: 1 mass, 2 dev, 4 graddiv, 8 G/D, 16 C, 32 advection; 63 = all */
    int apply_bc;    /* 1: Dirichlet elimination; 0: natural boundaries everywhere */
    int vms_dt_coupling; /* 1: add c_t*rho*tau_M*(V/4)*dN_a/dx_j to D (fluid) */
    int box_solid;   /* box only: 1 = every element is solid */
    double y_h;      /* Y: voxel spacing */
    double y_rd;     /* Y: daughter radius / parent radius */
    double y_ld;     /* Y: daughter length (parent length is L) */
    double y_th1, y_th2; /* Y: daughter angles from the z axis (radians), toward +x and -x */
    double u_max;    /* centreline speed of the advective Poiseuille state (0 = at rest) */
} synth_params;

typedef struct {
    int64_t n_phys, n_b, nnzb, n_tets, nnz_L, n_iface;
    int S, nzn;                 /* section nodes per side, axial node layers */
    int32_t *blk_of_phys, *virt_of_phys;
    uint8_t *node_kind;         /* per block row: 0 fluid, 1 solid, 2 interface (phys), 3 virtual */
    double *xyz;                /* per block row */
    double *xyz_phys;
    int32_t *rp, *ci; double *val;     /* K: 4x4 BSR */
    uint8_t *mask;              /* 4 per block row, 1 = Dirichlet dof */
    int32_t *Lrp, *Lci; double *Lval; uint8_t *Lmask;
    int32_t *tv, *tp; uint8_t *tsolid;
    double *uadv;               /* advective velocity per block row (3; zero off the fluid) */
    int n_out;                  /* outlets; entries of outlet k are out_off[k] .. out_off[k+1]-1 */
    int64_t *out_off; int32_t *out_blk; double *out_a;   /* block row and a (3) per entry */
} synth_sys;

/* ---- counter-based generator (Vigna's splitmix64 output function) ---- */
static uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

/* Uniform[-1,1) per entry i: (u >> 11) * 2^-53 * 2 - 1, u = splitmix64(seed ^ i*C). Masked
 * entries (mask[i] != 0) are set to zero.  mask may be NULL. */
void synth_rhs(uint64_t seed, int64_t n, const uint8_t* mask, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        uint64_t u = sm64(seed ^ ((uint64_t)i * 0xD1B54A32D192ED03ULL));
        double v = (double)(u >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
        out[i] = (mask && mask[i]) ? 0.0 : v;
    }
}

/* First-order generalized-alpha parameters from the spectral radius (Sec. 3.4). */
void synth_genalpha(double rho_inf, double* am, double* af, double* g) {
    *am = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf);
    *af = 1.0 / (1.0 + rho_inf);
    *g = 1.0 / (1.0 + rho_inf);
}

/* ---- element geometry ---- */
static double tet_grad(const double* x, double dN[4][3]) {
    double J[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) J[i][k] = x[3 * (k + 1) + i] - x[i];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    /* inverse: Ji[k][i] = d xi_k / d x_i */
    double Ji[3][3];
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int i = 0; i < 3; ++i) {
        dN[1][i] = Ji[0][i]; dN[2][i] = Ji[1][i]; dN[3][i] = Ji[2][i];
        dN[0][i] = -(Ji[0][i] + Ji[1][i] + Ji[2][i]);
    }
    return det;
}

/* tau_M and tau_C of the fluid VMS (Sec. 3.2) for the advective velocity ub (NULL = at rest). */
static void fluid_tau(const double* x, const synth_params* p, const double* ub, double* tauM, double* tauC) {
    double dN[4][3];
    tet_grad(x, dN);
    const double c = cbrt(2.0) / 2.0;
    const double M[3][3] = {{2 * c, c, c}, {c, 2 * c, c}, {c, c, 2 * c}};
    double G[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) s += dN[k + 1][i] * M[k][l] * dN[l + 1][j];
            G[i][j] = s;
        }
    double GG = 0.0, trG = 0.0, uGu = 0.0;
    for (int i = 0; i < 3; ++i) {
        trG += G[i][i];
        for (int j = 0; j < 3; ++j) {
            GG += G[i][j] * G[i][j];
            if (ub) uGu += ub[i] * G[i][j] * ub[j];
        }
    }
    const double CT = 4.0, CI = 36.0;
    double nu = p->mu_f / p->rho_f;
    *tauM = 1.0 / p->rho_f / sqrt(CT / (p->dt * p->dt) + uGu + CI * nu * nu * GG);
    *tauC = 1.0 / (*tauM * trG);
}

/* Element matrix, 16x16, index 4*a + c (c = 0,1,2 velocity, 3 pressure). u4: the advective
 * velocity at the 4 vertices (12 values) or NULL (at rest); ignored for solid elements.
 * Returns the volume. */
static double element_matrix(const double* x, const double* u4, const synth_params* p, int solid, double* Ke) {
    double dN[4][3];
    double det = tet_grad(x, dN);
    double V = fabs(det) / 6.0;
    double am, af, g;
    synth_genalpha(p->rho_inf, &am, &af, &g);
    double ct = am / (af * g * p->dt);
    memset(Ke, 0, sizeof(double) * 256);
    double rho, visc, gd = 0.0, tauM = 0.0, tauC = 0.0;
    int conv = !solid && u4 != NULL && (p->terms & 32);
    double ub[3] = {0.0, 0.0, 0.0}, gu[3][3] = {{0.0}};   /* centroid velocity, grad u (d u_i / d x_j) */
    if (conv)
        for (int i = 0; i < 3; ++i) {
            ub[i] = 0.25 * (u4[i] + u4[3 + i] + u4[6 + i] + u4[9 + i]);
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 4; ++c) gu[i][j] += u4[3 * c + i] * dN[c][j];
        }
    if (!solid) {
        fluid_tau(x, p, conv ? ub : NULL, &tauM, &tauC);
        rho = p->rho_f; visc = p->mu_f; gd = tauC;
    } else {
        double mu_s = p->E_s / (2.0 * (1.0 + p->nu_s));
        rho = p->rho_s; visc = (af * g * p->dt / am) * mu_s;
    }
    double kappa = p->E_s / (3.0 * (1.0 - 2.0 * p->nu_s));
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double Mab = V * (a == b ? 2.0 : 1.0) / 20.0;
            double Lab = V * (dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2]);
            double ua = ub[0] * dN[a][0] + ub[1] * dN[a][1] + ub[2] * dN[a][2];   /* ub . grad N_a */
            double uB = ub[0] * dN[b][0] + ub[1] * dN[b][1] + ub[2] * dN[b][2];   /* ub . grad N_b */
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double v = 0.0;
                    if (p->terms & 1) v += (i == j) ? rho * ct * Mab : 0.0;
                    if (p->terms & 2)
                        v += visc * ((i == j ? Lab : 0.0) + V * dN[a][j] * dN[b][i]
                                     - (2.0 / 3.0) * V * dN[a][i] * dN[b][j]);
                    if (p->terms & 4) v += gd * V * dN[a][i] * dN[b][j];
                    if (conv) {
                        if (i == j) v += rho * (V / 4.0) * uB + tauM * rho * rho * ua * (ct * (V / 4.0) + V * uB);
                        v += rho * Mab * gu[i][j];
                    }
                    Ke[(4 * a + i) * 16 + 4 * b + j] = v;
                }
            for (int i = 0; i < 3; ++i) {
                double gv = 0.0, dv = 0.0;
                if (p->terms & 8) {
                    gv = -(V / 4.0) * dN[a][i];             /* G[(a,i), b] */
                    dv = (V / 4.0) * dN[b][i];              /* D[a, (b,i)] = -G[(b,i), a] at rest */
                    if (!solid && p->vms_dt_coupling) dv += ct * rho * tauM * (V / 4.0) * dN[a][i];
                }
                if (conv) {
                    gv += tauM * rho * V * ua * dN[b][i];
                    dv += tauM * rho * V * dN[a][i] * uB;
                }
                Ke[(4 * a + i) * 16 + 4 * b + 3] = gv;
                Ke[(4 * a + 3) * 16 + 4 * b + i] = dv;
            }
            if (p->terms & 16)
                Ke[(4 * a + 3) * 16 + 4 * b + 3] = solid ? (ct / kappa) * Mab : tauM * Lab;
        }
    return V;
}

/* Test hooks: element matrix and tau of one tetrahedron given its 4 vertices (12 doubles) and
 * optionally the advective velocity at them (u4, 12 doubles, or NULL). */
double synth_element(const double* x4, const double* u4, const synth_params* p, int solid, double* Ke) {
    return element_matrix(x4, u4, p, solid, Ke);
}
void synth_tau(const double* x4, const double* ub, const synth_params* p, double* tauM, double* tauC) {
    fluid_tau(x4, p, ub, tauM, tauC);
}

/* ---- geometry helpers ---- */
static double shell_radius(const synth_params* p, int s) {
    int mf = p->m_core + p->n_bl;
    double S = 0.0, f = 1.0;
    for (int t = 0; t < p->n_bl; ++t) { S += f; f *= p->bl_ratio; }
    double rc = p->R / (1.0 + S / p->m_core);
    double hc = rc / p->m_core;
    if (s <= p->m_core) return s * hc;
    if (s <= mf) {
        double r = rc; f = 1.0;
        for (int t = 0; t < s - p->m_core; ++t) { r += hc * f; f *= p->bl_ratio; }
        return (s == mf) ? p->R : r;
    }
    return p->R + (s - mf) * (p->wall_ratio - 1.0) * p->R / p->n_wall;
}

static void section_xy(const synth_params* p, int m, int i, int j, double* x, double* y, int* shell) {
    int dx = i - m, dy = j - m;
    int s = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    *shell = s;
    if (s == 0) { *x = 0.0; *y = 0.0; return; }
    double t;
    if (dx == s) t = dy;
    else if (dy == s) t = 2 * s - dx;
    else if (dx == -s) t = 4 * s - dy;
    else t = 6 * s + dx;
    if (t < 0) t += 8 * s;
    double th = 2.0 * M_PI * t / (8.0 * s);
    double r = shell_radius(p, s);
    *x = r * cos(th); *y = r * sin(th);
}

static int find_col(const int32_t* ci, int32_t lo, int32_t hi, int32_t c) {
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (ci[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}

#define ROWCAP 64
static int row_insert(int32_t* cols, uint8_t* cnt, int64_t r, int32_t c) {
    int32_t* row = cols + r * ROWCAP;
    for (int t = 0; t < cnt[r]; ++t) if (row[t] == c) return 0;
    if (cnt[r] >= ROWCAP) return -1;
    row[cnt[r]++] = c;
    return 0;
}
static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* ---- Y-bifurcation geometry ---- */
typedef struct {
    double a[3], u[3];  /* branch start and unit direction */
    double len, r;      /* length and lumen radius */
    int cap_at_end;     /* 1: spherical cap at the far end (parent), 0: at the start (daughters) */
} y_branch;

static void y_branches(const synth_params* p, y_branch b[3]) {
    double R = p->R, rd = p->y_rd * p->R;
    y_branch* q = &b[0];
    q->a[0] = 0.0; q->a[1] = 0.0; q->a[2] = -p->L; q->u[0] = 0.0; q->u[1] = 0.0; q->u[2] = 1.0;
    q->len = p->L; q->r = R; q->cap_at_end = 1;
    for (int d = 0; d < 2; ++d) {
        q = &b[1 + d];
        double th = d == 0 ? p->y_th1 : p->y_th2, sg = d == 0 ? 1.0 : -1.0;
        q->a[0] = q->a[1] = q->a[2] = 0.0;
        q->u[0] = sg * sin(th); q->u[1] = 0.0; q->u[2] = cos(th);
        q->len = p->y_ld; q->r = rd; q->cap_at_end = 0;
    }
}

/* distance from x to branch q relative to its radius; a large value outside the free-end cut */
static double y_rel(const y_branch* q, const double* x) {
    double d[3] = {x[0] - q->a[0], x[1] - q->a[1], x[2] - q->a[2]};
    double t = d[0] * q->u[0] + d[1] * q->u[1] + d[2] * q->u[2];
    if (q->cap_at_end ? t < 0.0 : t > q->len) return 1e30;
    if (q->cap_at_end ? t > q->len : t < 0.0) {
        double c = q->cap_at_end ? q->len : 0.0;
        double e[3] = {d[0] - c * q->u[0], d[1] - c * q->u[1], d[2] - c * q->u[2]};
        return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) / q->r;
    }
    double e[3] = {d[0] - t * q->u[0], d[1] - t * q->u[1], d[2] - t * q->u[2]};
    return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) / q->r;
}
static double y_min_rel(const y_branch b[3], const double* x) {
    double m = 1e30;
    for (int k = 0; k < 3; ++k) { double v = y_rel(&b[k], x); if (v < m) m = v; }
    return m;
}

/* Voxels, nodes, tetrahedra and Dirichlet flags of the Y (mode 2).  Fills the mesh part of s;
 * vdir / mdir get one flag per physical node. */
static int build_y(const synth_params* p, synth_sys* s, uint8_t** vdir_out, uint8_t** mdir_out) {
    y_branch br[3];
    y_branches(p, br);
    double h = p->y_h, W = p->wall_ratio;
    double lo[3] = {-W * p->R, -W * p->R, -p->L}, hi[3] = {W * p->R, W * p->R, 0.0};
    for (int d = 1; d < 3; ++d) {
        double ew = W * br[d].r;
        for (int c = 0; c < 3; ++c) {
            double e = br[d].a[c] + br[d].len * br[d].u[c];
            if (e - ew < lo[c]) lo[c] = e - ew;
            if (e + ew > hi[c]) hi[c] = e + ew;
        }
    }
    lo[2] = -p->L;   /* the inlet plane is a grid plane */
    int nc[3];
    for (int c = 0; c < 3; ++c) nc[c] = (int)ceil((hi[c] - lo[c]) / h) + 1;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t ngn = (int64_t)(nc[0] + 1) * (nc[1] + 1) * (nc[2] + 1);
    if (ngn > INT32_MAX) return -2;
    uint8_t* keep = (uint8_t*)calloc(ncell, 1);
    int32_t* gid = (int32_t*)malloc(sizeof(int32_t) * ngn);
    if (!keep || !gid) { free(keep); free(gid); return -3; }
    for (int64_t g = 0; g < ngn; ++g) gid[g] = -1;
    int64_t nx1 = nc[0] + 1, nxy1 = (int64_t)(nc[0] + 1) * (nc[1] + 1);
    int64_t nkept = 0;
    for (int k = 0; k < nc[2]; ++k)
        for (int j = 0; j < nc[1]; ++j)
            for (int i = 0; i < nc[0]; ++i) {
                double x[3] = {lo[0] + (i + 0.5) * h, lo[1] + (j + 0.5) * h, lo[2] + (k + 0.5) * h};
                if (y_min_rel(br, x) < W) {
                    keep[i + (int64_t)nc[0] * (j + (int64_t)nc[1] * k)] = 1;
                    ++nkept;
                    for (int c = 0; c < 8; ++c)
                        gid[(i + (c & 1)) + nx1 * (j + ((c >> 1) & 1)) + nxy1 * (k + (c >> 2))] = 0;
                }
            }
    /* physical nodes in grid order */
    int64_t n_phys = 0;
    for (int64_t g = 0; g < ngn; ++g) if (gid[g] == 0) gid[g] = (int32_t)n_phys++;
    s->n_phys = n_phys; s->S = nc[0] + 1; s->nzn = nc[2] + 1;
    s->xyz_phys = (double*)malloc(sizeof(double) * 3 * n_phys);
    int32_t* gk = (int32_t*)malloc(sizeof(int32_t) * n_phys);
    for (int64_t g = 0; g < ngn; ++g)
        if (gid[g] >= 0) {
            int64_t n = gid[g];
            int i = (int)(g % nx1), j = (int)((g / nx1) % (nc[1] + 1)), k = (int)(g / nxy1);
            s->xyz_phys[3 * n] = lo[0] + i * h; s->xyz_phys[3 * n + 1] = lo[1] + j * h;
            s->xyz_phys[3 * n + 2] = lo[2] + k * h;
            gk[n] = k;
        }
    /* tetrahedra (physical vertex ids for now) and their fluid/solid class */
    s->n_tets = 6 * nkept;
    s->tv = (int32_t*)malloc(sizeof(int32_t) * 4 * s->n_tets);
    s->tp = (int32_t*)malloc(sizeof(int32_t) * 4 * s->n_tets);
    s->tsolid = (uint8_t*)malloc(s->n_tets);
    uint8_t* touch = (uint8_t*)calloc(n_phys, 1);   /* bit 1: fluid tet, bit 2: solid tet */
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t t = 0;
    for (int k = 0; k < nc[2]; ++k)
        for (int j = 0; j < nc[1]; ++j)
            for (int i = 0; i < nc[0]; ++i) {
                if (!keep[i + (int64_t)nc[0] * (j + (int64_t)nc[1] * k)]) continue;
                for (int q = 0; q < 6; ++q) {
                    int off[4][3] = {{0, 0, 0}};
                    int cur[3] = {0, 0, 0};
                    for (int st = 0; st < 3; ++st) {
                        cur[perm[q][st]] = 1;
                        off[st + 1][0] = cur[0]; off[st + 1][1] = cur[1]; off[st + 1][2] = cur[2];
                    }
                    int32_t v[4];
                    double x[12], cen[3] = {0.0, 0.0, 0.0};
                    for (int a = 0; a < 4; ++a) {
                        v[a] = gid[(i + off[a][0]) + nx1 * (j + off[a][1]) + nxy1 * (k + off[a][2])];
                        memcpy(x + 3 * a, s->xyz_phys + 3 * (int64_t)v[a], 3 * sizeof(double));
                        for (int c = 0; c < 3; ++c) cen[c] += 0.25 * x[3 * a + c];
                    }
                    double dN[4][3];
                    if (tet_grad(x, dN) < 0.0) { int32_t tmp = v[2]; v[2] = v[3]; v[3] = tmp; }
                    int solid = !(y_min_rel(br, cen) < 1.0);
                    for (int a = 0; a < 4; ++a) { s->tv[4 * t + a] = v[a]; touch[v[a]] |= (uint8_t)(solid ? 2 : 1); }
                    s->tsolid[t] = (uint8_t)solid;
                    ++t;
                }
            }
    free(keep); free(gid);
    /* block numbering: each interface node followed by its virtual (pressure) node */
    s->blk_of_phys = (int32_t*)malloc(sizeof(int32_t) * n_phys);
    s->virt_of_phys = (int32_t*)malloc(sizeof(int32_t) * n_phys);
    int64_t nb = 0, nif = 0;
    for (int64_t n = 0; n < n_phys; ++n) {
        s->blk_of_phys[n] = (int32_t)nb++;
        if (touch[n] == 3) { s->virt_of_phys[n] = (int32_t)nb++; ++nif; }
        else s->virt_of_phys[n] = -1;
    }
    s->n_b = nb; s->n_iface = nif;
    s->node_kind = (uint8_t*)malloc(nb);
    s->xyz = (double*)malloc(sizeof(double) * 3 * nb);
    for (int64_t n = 0; n < n_phys; ++n) {
        int32_t b = s->blk_of_phys[n];
        s->node_kind[b] = (uint8_t)(touch[n] == 1 ? 0 : (touch[n] == 2 ? 1 : 2));
        memcpy(s->xyz + 3 * b, s->xyz_phys + 3 * n, 3 * sizeof(double));
        if (s->virt_of_phys[n] >= 0) {
            int32_t vv = s->virt_of_phys[n];
            s->node_kind[vv] = 3;
            memcpy(s->xyz + 3 * vv, s->xyz_phys + 3 * n, 3 * sizeof(double));
        }
    }
    for (int64_t e = 0; e < s->n_tets; ++e)
        for (int a = 0; a < 4; ++a) {
            int32_t n = s->tv[4 * e + a];
            s->tv[4 * e + a] = s->blk_of_phys[n];
            s->tp[4 * e + a] = (s->tsolid[e] && s->virt_of_phys[n] >= 0) ? s->virt_of_phys[n] : s->blk_of_phys[n];
        }
    /* Dirichlet flags */
    uint8_t* vdir = (uint8_t*)calloc(n_phys, 1);
    uint8_t* mdir = (uint8_t*)calloc(n_phys, 1);
    for (int64_t n = 0; n < n_phys; ++n) {
        const double* x = s->xyz_phys + 3 * n;
        int outlet = 0;
        for (int d = 1; d < 3; ++d) {
            double dd[3] = {x[0] - br[d].a[0], x[1] - br[d].a[1], x[2] - br[d].a[2]};
            double tt = dd[0] * br[d].u[0] + dd[1] * br[d].u[1] + dd[2] * br[d].u[2];
            double e[3] = {dd[0] - tt * br[d].u[0], dd[1] - tt * br[d].u[1], dd[2] - tt * br[d].u[2]};
            double rr = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            if (tt > br[d].len - h && rr < W * br[d].r + h) outlet = 1;
        }
        int inlet = gk[n] == 0;
        vdir[n] = (uint8_t)(inlet || (outlet && (touch[n] & 2)));
        mdir[n] = (uint8_t)(inlet || outlet || (touch[n] & 2));
    }
    free(touch); free(gk);
    *vdir_out = vdir; *mdir_out = mdir;
    return 0;
}

void synth_free(synth_sys* s) {
    if (!s) return;
    free(s->blk_of_phys); free(s->virt_of_phys); free(s->node_kind); free(s->xyz); free(s->xyz_phys);
    free(s->rp); free(s->ci); free(s->val); free(s->mask);
    free(s->Lrp); free(s->Lci); free(s->Lval); free(s->Lmask);
    free(s->tv); free(s->tp); free(s->tsolid);
    free(s->uadv); free(s->out_off); free(s->out_blk); free(s->out_a);
    free(s);
}

/* Build the system.  Returns 0 on success, <0 on failure. */
/* Mesh of the tube (mode 0) and box (mode 1): fills the mesh part of s and the Dirichlet flags. */
static int build_structured(const synth_params* p, synth_sys* s, uint8_t** vdir_out, uint8_t** mdir_out) {
    int box = (p->mode == 1);
    int m = box ? 0 : p->m_core + p->n_bl + p->n_wall;
    int mf = p->m_core + p->n_bl;
    int Sx = box ? p->m_core + 1 : 2 * m + 1;   /* nodes along i */
    int Sy = box ? p->n_bl + 1 : 2 * m + 1;     /* nodes along j */
    int nzn = p->nz + 1;
    int has_wall = (!box && p->n_wall > 0);
    int64_t n_phys = (int64_t)Sx * Sy * nzn;
    s->n_phys = n_phys; s->S = Sx; s->nzn = nzn;
    int* shell = (int*)malloc(sizeof(int) * n_phys);
    s->xyz_phys = (double*)malloc(sizeof(double) * 3 * n_phys);
    for (int k = 0; k < nzn; ++k)
        for (int j = 0; j < Sy; ++j)
            for (int i = 0; i < Sx; ++i) {
                int64_t n = i + (int64_t)Sx * (j + (int64_t)Sy * k);
                double x, y; int sh;
                if (box) { x = i * p->R; y = j * p->R; sh = 0; }
                else section_xy(p, m, i, j, &x, &y, &sh);
                shell[n] = sh;
                s->xyz_phys[3 * n] = x; s->xyz_phys[3 * n + 1] = y;
                s->xyz_phys[3 * n + 2] = box ? k * p->R : k * p->L / p->nz;
            }
    /* block numbering: physical nodes in order, each interface node followed by its virtual node */
    s->blk_of_phys = (int32_t*)malloc(sizeof(int32_t) * n_phys);
    s->virt_of_phys = (int32_t*)malloc(sizeof(int32_t) * n_phys);
    int64_t nb = 0, nif = 0;
    for (int64_t n = 0; n < n_phys; ++n) {
        s->blk_of_phys[n] = (int32_t)nb++;
        if (has_wall && shell[n] == mf) { s->virt_of_phys[n] = (int32_t)nb++; ++nif; }
        else s->virt_of_phys[n] = -1;
    }
    s->n_b = nb; s->n_iface = nif;
    s->node_kind = (uint8_t*)malloc(nb);
    s->xyz = (double*)malloc(sizeof(double) * 3 * nb);
    for (int64_t n = 0; n < n_phys; ++n) {
        int32_t b = s->blk_of_phys[n];
        s->node_kind[b] = box ? (uint8_t)(p->box_solid ? 1 : 0)
                              : (uint8_t)(has_wall ? (shell[n] < mf ? 0 : (shell[n] == mf ? 2 : 1)) : 0);
        memcpy(s->xyz + 3 * b, s->xyz_phys + 3 * n, 3 * sizeof(double));
        if (s->virt_of_phys[n] >= 0) {
            int32_t v = s->virt_of_phys[n];
            s->node_kind[v] = 3;
            memcpy(s->xyz + 3 * v, s->xyz_phys + 3 * n, 3 * sizeof(double));
        }
    }
    /* tetrahedra */
    int ncx = Sx - 1, ncy = Sy - 1;
    int64_t ncell = (int64_t)ncx * ncy * p->nz;
    s->n_tets = 6 * ncell;
    s->tv = (int32_t*)malloc(sizeof(int32_t) * 4 * s->n_tets);
    s->tp = (int32_t*)malloc(sizeof(int32_t) * 4 * s->n_tets);
    s->tsolid = (uint8_t*)malloc(s->n_tets);
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t t = 0;
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < ncy; ++j)
            for (int i = 0; i < ncx; ++i) {
                int fi = (!box && i < m) ? 1 : 0, fj = (!box && j < m) ? 1 : 0;
                int smax = 0;
                for (int c = 0; c < 4; ++c) {
                    int64_t n = (i + (c & 1)) + (int64_t)Sx * ((j + (c >> 1)) + (int64_t)Sy * k);
                    if (shell[n] > smax) smax = shell[n];
                }
                int solid = box ? p->box_solid : (has_wall && smax > mf);
                for (int q = 0; q < 6; ++q) {
                    int off[4][3] = {{0, 0, 0}};
                    int cur[3] = {0, 0, 0};
                    for (int st = 0; st < 3; ++st) {
                        cur[perm[q][st]] = 1;
                        off[st + 1][0] = cur[0]; off[st + 1][1] = cur[1]; off[st + 1][2] = cur[2];
                    }
                    int64_t v[4];
                    for (int a = 0; a < 4; ++a) {
                        int ii = i + (fi ? 1 - off[a][0] : off[a][0]);
                        int jj = j + (fj ? 1 - off[a][1] : off[a][1]);
                        int kk = k + off[a][2];
                        v[a] = ii + (int64_t)Sx * (jj + (int64_t)Sy * kk);
                    }
                    double x[12];
                    for (int a = 0; a < 4; ++a) memcpy(x + 3 * a, s->xyz_phys + 3 * v[a], 3 * sizeof(double));
                    double dN[4][3];
                    if (tet_grad(x, dN) < 0.0) { int64_t tmp = v[2]; v[2] = v[3]; v[3] = tmp; }
                    for (int a = 0; a < 4; ++a) {
                        s->tv[4 * t + a] = s->blk_of_phys[v[a]];
                        s->tp[4 * t + a] = (solid && s->virt_of_phys[v[a]] >= 0) ? s->virt_of_phys[v[a]]
                                                                                : s->blk_of_phys[v[a]];
                    }
                    s->tsolid[t] = (uint8_t)solid;
                    ++t;
                }
            }
    /* Dirichlet flags per physical node */
    uint8_t* vdir = (uint8_t*)calloc(n_phys, 1);
    uint8_t* mdir = (uint8_t*)calloc(n_phys, 1);
    for (int64_t n = 0; n < n_phys; ++n) {
        int k = (int)(n / ((int64_t)Sx * Sy));
        int sh = shell[n];
        if (box) {
            int64_t rem = n % ((int64_t)Sx * Sy);
            int i = (int)(rem % Sx), j = (int)(rem / Sx);
            int side = (i == 0 || i == Sx - 1 || j == 0 || j == Sy - 1);
            vdir[n] = (uint8_t)(side || k == 0);
            mdir[n] = (uint8_t)(side || k == 0 || k == p->nz);
        } else {
            vdir[n] = (uint8_t)(!has_wall ? ((sh == m) || (k == 0)) : ((k == 0) || (sh >= mf && k == p->nz)));
            mdir[n] = (uint8_t)((sh >= mf) || k == 0 || k == p->nz);
        }
    }
    free(shell);
    *vdir_out = vdir; *mdir_out = mdir;
    return 0;
}

int synth_build(const synth_params* p, synth_sys** out) {
    synth_sys* s = (synth_sys*)calloc(1, sizeof(synth_sys));
    uint8_t *vdir = NULL, *mdir = NULL;
    int rc = p->mode == 2 ? build_y(p, s, &vdir, &mdir) : build_structured(p, s, &vdir, &mdir);
    if (rc != 0) { free(vdir); free(mdir); synth_free(s); return rc; }
    int64_t nb = s->n_b, n_phys = s->n_phys;
    /* K pattern */
    int32_t* cols = (int32_t*)malloc(sizeof(int32_t) * ROWCAP * nb);
    uint8_t* cnt = (uint8_t*)calloc(nb, 1);
    int bad = 0;
    for (int64_t b = 0; b < nb; ++b) bad |= row_insert(cols, cnt, b, (int32_t)b);
    for (int64_t e = 0; e < s->n_tets && !bad; ++e) {
        const int32_t* va = s->tv + 4 * e; const int32_t* pa = s->tp + 4 * e;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                bad |= row_insert(cols, cnt, va[a], va[b]);
                bad |= row_insert(cols, cnt, va[a], pa[b]);
                bad |= row_insert(cols, cnt, pa[a], va[b]);
                bad |= row_insert(cols, cnt, pa[a], pa[b]);
            }
    }
    if (bad) { free(cols); free(cnt); free(vdir); free(mdir); synth_free(s); return -1; }
    s->rp = (int32_t*)malloc(sizeof(int32_t) * (nb + 1));
    s->rp[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        qsort(cols + b * ROWCAP, cnt[b], sizeof(int32_t), cmp_i32);
        s->rp[b + 1] = s->rp[b] + cnt[b];
    }
    s->nnzb = s->rp[nb];
    s->ci = (int32_t*)malloc(sizeof(int32_t) * s->nnzb);
    for (int64_t b = 0; b < nb; ++b) memcpy(s->ci + s->rp[b], cols + b * ROWCAP, sizeof(int32_t) * cnt[b]);
    s->val = (double*)calloc((size_t)s->nnzb * 16, sizeof(double));
    /* advective state: Poiseuille profile on the fluid block rows (tube and box) */
    s->uadv = (double*)calloc(3 * (size_t)nb, sizeof(double));
    int conv = p->u_max != 0.0 && p->mode != 2;
    if (conv) {
        double cx = 0.0, cy = 0.0, R = p->R;
        if (p->mode == 1) {
            double lx = (double)(s->S - 1) * p->R, ly = (double)(n_phys / ((int64_t)s->S * s->nzn) - 1) * p->R;
            cx = 0.5 * lx; cy = 0.5 * ly; R = 0.5 * (lx < ly ? lx : ly);
        }
        for (int64_t b = 0; b < nb; ++b) {
            if (s->node_kind[b] == 1 || s->node_kind[b] == 3) continue;
            double dx = s->xyz[3 * b] - cx, dy = s->xyz[3 * b + 1] - cy;
            double w = 1.0 - (dx * dx + dy * dy) / (R * R);
            s->uadv[3 * b + 2] = w > 0.0 ? p->u_max * w : 0.0;
        }
    }
    /* assemble */
    double Ke[256];
    for (int64_t e = 0; e < s->n_tets; ++e) {
        const int32_t* va = s->tv + 4 * e; const int32_t* pa = s->tp + 4 * e;
        double x[12], u4[12];
        for (int a = 0; a < 4; ++a) {
            memcpy(x + 3 * a, s->xyz + 3 * va[a], 3 * sizeof(double));
            memcpy(u4 + 3 * a, s->uadv + 3 * va[a], 3 * sizeof(double));
        }
        element_matrix(x, conv ? u4 : NULL, p, s->tsolid[e], Ke);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                /* A part: (va[a], va[b]) [i][j]; G: (va[a], pa[b]) [i][3]; D: (pa[a], va[b]) [3][j]; C: (pa[a], pa[b]) [3][3] */
                int32_t r, c, pos;
                r = va[a]; c = va[b]; pos = find_col(s->ci, s->rp[r], s->rp[r + 1], c);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) s->val[16 * (int64_t)pos + 4 * i + j] += Ke[(4 * a + i) * 16 + 4 * b + j];
                c = pa[b]; pos = find_col(s->ci, s->rp[r], s->rp[r + 1], c);
                for (int i = 0; i < 3; ++i) s->val[16 * (int64_t)pos + 4 * i + 3] += Ke[(4 * a + i) * 16 + 4 * b + 3];
                r = pa[a]; c = va[b]; pos = find_col(s->ci, s->rp[r], s->rp[r + 1], c);
                for (int j = 0; j < 3; ++j) s->val[16 * (int64_t)pos + 12 + j] += Ke[(4 * a + 3) * 16 + 4 * b + j];
                c = pa[b]; pos = find_col(s->ci, s->rp[r], s->rp[r + 1], c);
                s->val[16 * (int64_t)pos + 15] += Ke[(4 * a + 3) * 16 + 4 * b + 3];
            }
    }
    /* Dirichlet mask (velocity dofs only) */
    s->mask = (uint8_t*)calloc(4 * nb, 1);
    if (p->apply_bc) {
        for (int64_t n = 0; n < n_phys; ++n)
            if (vdir[n]) for (int c = 0; c < 3; ++c) s->mask[4 * s->blk_of_phys[n] + c] = 1;
        for (int64_t n = 0; n < n_phys; ++n)
            if (s->virt_of_phys[n] >= 0)
                for (int c = 0; c < 3; ++c) s->mask[4 * s->virt_of_phys[n] + c] = 1;
        for (int64_t r = 0; r < nb; ++r)
            for (int32_t q = s->rp[r]; q < s->rp[r + 1]; ++q) {
                int32_t c = s->ci[q];
                double* blk = s->val + 16 * (int64_t)q;
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j)
                        if (s->mask[4 * r + i] || s->mask[4 * (int64_t)c + j]) blk[4 * i + j] = 0.0;
                if (c == r)
                    for (int i = 0; i < 4; ++i) if (s->mask[4 * r + i]) blk[5 * i] = 1.0;
            }
    } else {
        /* virtual nodes still carry identity velocity rows */
        for (int64_t n = 0; n < n_phys; ++n)
            if (s->virt_of_phys[n] >= 0) {
                int32_t v = s->virt_of_phys[n];
                for (int c = 0; c < 3; ++c) s->mask[4 * v + c] = 1;
            }
        for (int64_t r = 0; r < nb; ++r)
            for (int32_t q = s->rp[r]; q < s->rp[r + 1]; ++q) {
                int32_t c = s->ci[q];
                double* blk = s->val + 16 * (int64_t)q;
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j)
                        if ((i < 3 && s->node_kind[r] == 3) || (j < 3 && s->node_kind[c] == 3)) blk[4 * i + j] = 0.0;
                if (c == r && s->node_kind[r] == 3) for (int i = 0; i < 3; ++i) blk[5 * i] = 1.0;
            }
    }
    /* outlet of the tube and box: faces of fluid elements on the plane z = z_max */
    s->out_off = (int64_t*)calloc(2, sizeof(int64_t));
    if (p->mode != 2) {
        double zmax = -INFINITY;
        for (int64_t n = 0; n < n_phys; ++n) if (s->xyz_phys[3 * n + 2] > zmax) zmax = s->xyz_phys[3 * n + 2];
        double* acc = (double*)calloc(nb, sizeof(double));
        static const int face[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        for (int64_t e = 0; e < s->n_tets; ++e) {
            if (s->tsolid[e]) continue;
            const int32_t* va = s->tv + 4 * e;
            for (int f = 0; f < 4; ++f) {
                const double* q[3];
                int on = 1;
                for (int t = 0; t < 3; ++t) {
                    q[t] = s->xyz + 3 * va[face[f][t]];
                    on &= q[t][2] == zmax;
                }
                if (!on) continue;
                double e1x = q[1][0] - q[0][0], e1y = q[1][1] - q[0][1];
                double e2x = q[2][0] - q[0][0], e2y = q[2][1] - q[0][1];
                double area = 0.5 * fabs(e1x * e2y - e1y * e2x);
                for (int t = 0; t < 3; ++t) acc[va[face[f][t]]] += area / 3.0;
            }
        }
        int64_t ne = 0;
        for (int64_t b = 0; b < nb; ++b) if (acc[b] != 0.0 && !s->mask[4 * b + 2]) ++ne;
        if (ne > 0) {
            s->n_out = 1;
            s->out_off[1] = ne;
            s->out_blk = (int32_t*)malloc(sizeof(int32_t) * ne);
            s->out_a = (double*)calloc(3 * (size_t)ne, sizeof(double));
            int64_t t = 0;
            for (int64_t b = 0; b < nb; ++b)
                if (acc[b] != 0.0 && !s->mask[4 * b + 2]) { s->out_blk[t] = (int32_t)b; s->out_a[3 * t + 2] = acc[b]; ++t; }
        }
        free(acc);
    }
    /* mesh-motion Laplacian over physical nodes, element factor 1/V:  entries dN_a . dN_b */
    {
        int32_t* lcols = cols;           /* reuse the scratch */
        memset(cnt, 0, nb);
        for (int64_t n = 0; n < n_phys; ++n) row_insert(lcols, cnt, n, (int32_t)n);
        int32_t* phys_of_blk = (int32_t*)malloc(sizeof(int32_t) * nb);
        for (int64_t n = 0; n < n_phys; ++n) phys_of_blk[s->blk_of_phys[n]] = (int32_t)n;
        for (int64_t e = 0; e < s->n_tets; ++e)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    row_insert(lcols, cnt, phys_of_blk[s->tv[4 * e + a]], phys_of_blk[s->tv[4 * e + b]]);
        s->Lrp = (int32_t*)malloc(sizeof(int32_t) * (n_phys + 1));
        s->Lrp[0] = 0;
        for (int64_t n = 0; n < n_phys; ++n) {
            qsort(lcols + n * ROWCAP, cnt[n], sizeof(int32_t), cmp_i32);
            s->Lrp[n + 1] = s->Lrp[n] + cnt[n];
        }
        s->nnz_L = s->Lrp[n_phys];
        s->Lci = (int32_t*)malloc(sizeof(int32_t) * s->nnz_L);
        for (int64_t n = 0; n < n_phys; ++n) memcpy(s->Lci + s->Lrp[n], lcols + n * ROWCAP, sizeof(int32_t) * cnt[n]);
        s->Lval = (double*)calloc(s->nnz_L, sizeof(double));
        for (int64_t e = 0; e < s->n_tets; ++e) {
            double x[12]; int32_t pn[4];
            for (int a = 0; a < 4; ++a) {
                pn[a] = phys_of_blk[s->tv[4 * e + a]];
                memcpy(x + 3 * a, s->xyz_phys + 3 * pn[a], 3 * sizeof(double));
            }
            double dN[4][3];
            tet_grad(x, dN);
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    int32_t pos = find_col(s->Lci, s->Lrp[pn[a]], s->Lrp[pn[a] + 1], pn[b]);
                    s->Lval[pos] += dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2];
                }
        }
        free(phys_of_blk);
        s->Lmask = (uint8_t*)calloc(n_phys, 1);
        if (p->apply_bc) {
            for (int64_t n = 0; n < n_phys; ++n) s->Lmask[n] = mdir[n];
            for (int64_t r = 0; r < n_phys; ++r)
                for (int32_t q = s->Lrp[r]; q < s->Lrp[r + 1]; ++q) {
                    int32_t c = s->Lci[q];
                    if (s->Lmask[r] || s->Lmask[c]) s->Lval[q] = (c == r) ? 1.0 : 0.0;
                }
        }
    }
    free(cols); free(cnt); free(vdir); free(mdir);
    *out = s;
    return 0;
}

void synth_info(const synth_sys* s, int64_t* info) {
    info[0] = s->n_phys; info[1] = s->n_b; info[2] = s->nnzb; info[3] = s->n_tets;
    info[4] = s->nnz_L; info[5] = s->n_iface; info[6] = s->S; info[7] = s->nzn;
    info[8] = s->n_out; info[9] = s->out_off[s->n_out];
}
void synth_get_flow(const synth_sys* s, double* uadv, int64_t* out_off, int32_t* out_blk, double* out_a) {
    memcpy(uadv, s->uadv, sizeof(double) * 3 * s->n_b);
    memcpy(out_off, s->out_off, sizeof(int64_t) * (s->n_out + 1));
    int64_t ne = s->out_off[s->n_out];
    if (ne) {
        memcpy(out_blk, s->out_blk, sizeof(int32_t) * ne);
        memcpy(out_a, s->out_a, sizeof(double) * 3 * ne);
    }
}
void synth_get_K(const synth_sys* s, int32_t* rp, int32_t* ci, double* val) {
    memcpy(rp, s->rp, sizeof(int32_t) * (s->n_b + 1));
    memcpy(ci, s->ci, sizeof(int32_t) * s->nnzb);
    memcpy(val, s->val, sizeof(double) * 16 * s->nnzb);
}
void synth_get_nodes(const synth_sys* s, double* xyz, uint8_t* mask, uint8_t* kind) {
    memcpy(xyz, s->xyz, sizeof(double) * 3 * s->n_b);
    memcpy(mask, s->mask, 4 * s->n_b);
    memcpy(kind, s->node_kind, s->n_b);
}
void synth_get_L(const synth_sys* s, int32_t* rp, int32_t* ci, double* val, uint8_t* mask, double* xyz) {
    memcpy(rp, s->Lrp, sizeof(int32_t) * (s->n_phys + 1));
    memcpy(ci, s->Lci, sizeof(int32_t) * s->nnz_L);
    memcpy(val, s->Lval, sizeof(double) * s->nnz_L);
    memcpy(mask, s->Lmask, s->n_phys);
    memcpy(xyz, s->xyz_phys, sizeof(double) * 3 * s->n_phys);
}
void synth_get_tets(const synth_sys* s, int32_t* tv, int32_t* tp, uint8_t* solid, int32_t* blk_of_phys) {
    memcpy(tv, s->tv, sizeof(int32_t) * 4 * s->n_tets);
    memcpy(tp, s->tp, sizeof(int32_t) * 4 * s->n_tets);
    memcpy(solid, s->tsolid, s->n_tets);
    memcpy(blk_of_phys, s->blk_of_phys, sizeof(int32_t) * s->n_phys);
}
