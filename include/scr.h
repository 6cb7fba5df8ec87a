/*
 * scr.h -- C ABI of the MI355X SCR+AMG linear-solve library (libscr.so).
 *
 * The library solves the two linear systems of every Newton corrector of the fully implicit
 * unified-continuum FSI method (Liu, Huang, Lu & Sun, arXiv 2206.06996):
 *
 *   (1) the 2x2 velocity/pressure block system  [A G; D C] [dv; dp] = b   (Sec. 3.5, the
 *       corrector linear system; the paper writes the blocks [A B; C D]), by flexible GMRES
 *       preconditioned with the Schur-complement-reduction preconditioner of Sec. 5.2.1 and
 *       Appendix B (Algorithm 1), whose Schur action is the matrix-free Algorithm 2.  GMRES
 *       on A is preconditioned by smoothed-aggregation AMG built on A; GMRES on the Schur
 *       complement by AMG built on the sparse approximation S^ = C - D diag(A)^-1 G
 *       (Sec. 5.2.1);
 *   (2) the mesh-motion system (harmonic extension, Sec. 2.2.2; solver of Sec. 5.2.2): CG
 *       preconditioned by AMG on a fixed Laplacian, three right-hand sides (x, y, z).
 *
 * Conventions (every function):
 *   - Pointers are DEVICE pointers (memory of the context's GPU) unless marked "host".
 *   - Inputs are borrowed for the duration of the call only; amg_setup copies what it keeps.
 *   - Calls enqueue work on `stream` (a hipStream_t passed as void*; NULL = the null stream)
 *     and return after that work has completed: Krylov control runs on the host.  Distinct
 *     handles may be used concurrently from different host threads on different streams.
 *     One handle must not be used by two threads at once.
 *   - No exception crosses the ABI.  Errors return a negative scr_status; scr_last_error()
 *     gives a message for the calling thread.  On error nothing is leaked.
 *   - Index arrays are 0-based int32; block values are row-major within a block; columns are
 *     strictly ascending within each block row; every block row stores its diagonal block.
 */
#ifndef SCR_H
#define SCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCR_OK = 0,
    SCR_NOT_CONVERGED = 1,     /* warning: x holds the last iterate, stats are filled */
    SCR_E_INVALID = -1,        /* malformed input (message in scr_last_error) */
    SCR_E_OOM = -2,            /* device allocation failed or the context budget is exceeded */
    SCR_E_HIP = -3,            /* HIP runtime error */
    SCR_E_BREAKDOWN = -4,      /* NaN/Inf in a Krylov recurrence */
    SCR_E_UNIMPLEMENTED = -5,
    SCR_E_NO_DEVICE = -6
} scr_status;

typedef enum { SCR_SYSTEM = 0, MESH_SYSTEM = 1 } scr_kind;
typedef enum { SCR_FP64 = 0, SCR_MIXED = 1, SCR_MIXED_FP32_INNER = 2 } scr_precision;
typedef enum { SCR_SMOOTH_JACOBI = 0, SCR_SMOOTH_CHEBYSHEV = 1 } scr_smoother;
/* AMG kind (amg_type): smoothed aggregation (default), or classical AMG with the settings of the
 * paper's table in Sec. 5.2 (see scr_amg_opts) */
typedef enum { SCR_AMG_SA = 0, SCR_AMG_CLASSICAL = 1 } scr_amg_type;

/* diagonal used in S^ (scr_amg_opts.schur_diag) */
typedef enum { SCR_DIAG_A = 0, SCR_DIAG_ABSROWSUM = 1 } scr_schur_diag;

/* outer preconditioner (scr_solve_opts.precond) */
typedef enum { SCR_PRECOND_SCR = 0, SCR_PRECOND_SIMPLE = 1 } scr_precond;

/* A square block-sparse matrix.  SCR_SYSTEM: bs = 4, block (i,j) = [[A_ij G_ij],[D_ij C_ij]]
 * with node-interleaved unknowns [vx vy vz p] (Sec. 3.5, corrector system; interface nodes
 * carry a duplicated pressure row as in Sec. 3.3, its velocity slots as identity rows).
 * MESH_SYSTEM: bs = 1, the scalar mesh Laplacian (the same operator acts on x, y and z). */
typedef struct {
    int32_t n_brows;
    int32_t bs;
    int64_t nnzb;
    const int32_t* row_ptr;    /* device, n_brows + 1 */
    const int32_t* col_idx;    /* device, nnzb */
    const double* val;         /* device, nnzb * bs * bs */
} scr_bsr;

/* Smoothed-aggregation AMG options (the paper uses BoomerAMG, Sec. 5.2 table of settings;
 * these are the SA replacements).  Defaults from scr_default_amg_opts. */
typedef struct {
    int precision;             /* SCR_FP64: everything in FP64.  SCR_MIXED: the AMG hierarchy values
                                  and the whole V-cycle in FP32 (cast at its entry and exit; the
                                  coarsest solve FP64); every Krylov level (the outer FGMRES, the A-
                                  and S-level solves of Algorithm 1, Algorithm 2's inner A solve), its
                                  Arnoldi process and Hessenberg least squares, the products with K,
                                  A, G, D, C and every true residual stay FP64.
                                  SCR_MIXED_FP32_INNER: as SCR_MIXED, and in addition Algorithm 2's
                                  inner A solve (GMRES to tol_I) runs on FP32 vectors with the FP32
                                  level-0 copy of A (dot products and updates accumulated in FP64,
                                  rounded on store; Hessenberg least squares FP64) */
    double theta;              /* strength threshold at level 0 (halved per level), 0.08 */
    int smoother;              /* scr_smoother, default Chebyshev */
    int cheb_degree;           /* 4 */
    double cheb_ratio;         /* lower end of the Chebyshev interval = lambda_hat / ratio, 30 */
    int jacobi_sweeps;         /* 2 */
    int coarse_max;            /* direct solve once a level has <= coarse_max unknowns, 1024 */
    int max_levels;            /* 10 */
    double max_coarse_ratio;   /* stop coarsening when n_{l+1} > ratio * n_l, 0.8 */
    uint64_t seed;             /* seed of the MIS-2 priorities, 0 */
    int schur_diag;            /* SCR_SYSTEM: the diagonal d in S^ = C - D d^-1 G (Sec. 5.2.1):
                                  SCR_DIAG_A (default) the diagonal of A; SCR_DIAG_ABSROWSUM the sums
                                  of the absolute values of A's rows (the SIMPLEC lumping) */
    int schur_cheb_degree;     /* SCR_SYSTEM: Chebyshev degree of AMG(S^); -1 (default): by the size of
                                  S^ (8 up to 1,000,000 rows, 12 up to 3,000,000, 16 above);
                                  0 = cheb_degree */
    double schur_cheb_ratio;   /* SCR_SYSTEM: Chebyshev interval ratio of AMG(S^), 100 (0 = cheb_ratio) */
    int amg_type;              /* SCR_AMG_SA (default) or SCR_AMG_CLASSICAL: the BoomerAMG settings of
                                  Sec. 5.2's table on the device.  Strength: row i depends on j (same
                                  function, i.e. the same velocity component for A's 3x3 blocks) when
                                  -s a_ij >= cl_theta max_k (-s a_ik), s = sign(a_ii).  HMIS: the
                                  Ruge-Stueben first pass inside domains of 256 consecutive rows (one
                                  workgroup each), then PMIS over the whole graph started from the
                                  first pass's C points whose strong connections stay in their domain
                                  (random part from splitmix64 of seed, level, row).  Extended+i
                                  interpolation truncated at trunc and to pmax entries per row (row
                                  sums kept).  Smoother: one hybrid Gauss-Seidel sweep before (forward)
                                  and after (backward) the coarse correction, Gauss-Seidel inside
                                  domains of 64 rows (one workgroup each), Jacobi between them; in
                                  its l1 form (l1_gs) each row's diagonal gains the absolute values
                                  of its couplings outside its domain, which keeps the sweep
                                  convergent for any symmetric positive definite matrix.
                                  Galerkin coarse operators, direct coarsest solve.  Any precision:
                                  the mixed forms run the V-cycle on FP32 copies of every level (the
                                  coarsest solve in FP64), as for smoothed aggregation.  The
                                  near-null space, theta, the smoother and Chebyshev fields are not
                                  used; amg_update sets the hierarchy up again.  The first
                                  agg_levels levels coarsen aggressively (two stages): HMIS gives
                                  first-stage C points; a second HMIS runs on the graph that joins
                                  two of them when one reaches the other through one or two strong
                                  dependencies; P is the truncated product P1 P2 of the extended+i
                                  interpolation P1 onto the first-stage C points and the extended+i
                                  interpolation P2 of P1^T A P1 onto the second-stage ones. */
    double cl_theta;           /* classical strength threshold, 0.5 */
    double trunc;              /* interpolation truncation factor, 0.3 */
    int pmax;                  /* interpolation entries per row, 5 (1..16) */
    int agg_levels;            /* classical: levels coarsened aggressively, 2 (0 = none; <= 16) */
    int l1_gs;                 /* classical: 1 (default) the l1 hybrid Gauss-Seidel, 0 the plain one */
} scr_amg_opts;

/* Krylov options.  Defaults: tol 1e-8 (outer), tol_A = tol_S = tol_I = 1e-3 and 200
 * iterations at every level (the paper's solver-settings table, Sec. 6), restart 50 for the
 * outer FGMRES and 30 for the inner GMRES levels; the mesh solve uses tol and max_it. */
typedef struct {
    double tol, tol_A, tol_S, tol_I;
    int max_it, max_it_A, max_it_S, max_it_I;
    int restart, restart_inner;
    int use_x0;                /* 1: x holds the initial guess on entry */
    int flexible_cg;           /* mesh solve: 1 = flexible CG (Notay), 0 = PCG; an FP32 hierarchy forces 1 */
    int precond;               /* scr_solve: SCR_PRECOND_SCR (default, Appendix B Algorithm 1) or
                                  SCR_PRECOND_SIMPLE (Sec. 5.2.1: S^ in place of S, d^-1 in the upper
                                  factor; SIMPLEC when the handle was set up with SCR_DIAG_ABSROWSUM) */
} scr_solve_opts;

typedef struct {
    int outer_it;              /* outer FGMRES iterations (or max mesh CG iterations) */
    int converged;
    double rel_res_true;       /* ||b - K x|| / ||b|| recomputed at exit (FP64) */
    int64_t calls_A, its_A;    /* Algorithm 1 steps 1 and 5 */
    int64_t calls_S, its_S;    /* Algorithm 1 step 3 */
    int64_t calls_I, its_I;    /* Algorithm 2 step 2 */
    int64_t vcycles_A, vcycles_S, vcycles_L;
    int64_t mesh_its[3];
    double mesh_rel[3];
    double t_setup_ms, t_solve_ms;
    int64_t device_bytes;      /* device memory held by the handle */
} scr_stats;

typedef struct scr_ctx scr_ctx;
typedef struct scr_handle scr_handle;

void scr_default_amg_opts(scr_amg_opts* o);        /* o: host */
void scr_default_solve_opts(scr_solve_opts* o);    /* o: host */

/* A context binds a device and an optional device-memory budget (bytes, 0 = unlimited) that
 * every handle created from it counts against.  Thread-safe. */
scr_status scr_ctx_create(int device, int64_t hbm_budget, scr_ctx** out /* host */);
void scr_ctx_destroy(scr_ctx* ctx);
int64_t scr_ctx_bytes_in_use(const scr_ctx* ctx);

/* Validate K and build everything the solves need (Sec. 5.2.1 for SCR_SYSTEM, Sec. 5.2.2 for
 * MESH_SYSTEM): for SCR_SYSTEM the block split A, G, D, C, the sparse Schur approximation S^,
 * AMG(A) with the six rigid-body modes of `coords` as near-null space, AMG(S^) with the
 * constant, and the Krylov workspaces; for MESH_SYSTEM AMG(L) with the constant.
 * coords: device, n_brows x 3 FP64 (node coordinates; required for SCR_SYSTEM, ignored for
 * MESH_SYSTEM).  K is copied.  Errors: SCR_E_INVALID for a malformed K (unsorted or
 * out-of-range columns, missing or zero diagonal, non-finite values, bs not 4/1 for the
 * kind) or for a sparse product of the setup (A P, R (A P)) with a row of more than 4,096
 * distinct block columns (a row coupled to nodes spread over the whole mesh), SCR_E_OOM,
 * SCR_E_HIP. */
scr_status amg_setup(scr_ctx* ctx, int kind, const scr_bsr* K, const double* coords,
                     const scr_amg_opts* opts /* host, NULL = defaults */, void* stream,
                     scr_handle** out /* host */);

/* Numeric re-setup for a new matrix on the same sparsity pattern (successive Newton correctors
 * and time steps, Sec. 3.5, change the values of the tangent matrix but not its pattern; the
 * mesh-motion matrix of Sec. 2.2.2 may be rescaled): K must have the handle's kind, n_brows,
 * nnzb, row_ptr and col_idx.  The strength flags, MIS-2 aggregates and every sparsity pattern of
 * both hierarchies are kept; every value-dependent quantity (the split, d and S^, the tentative
 * and smoothed prolongators, R, the Galerkin products, D^-1, lambda_hat, the coarse inverse, the
 * solve-phase copies) is recomputed exactly as amg_setup would from the same aggregates.
 * coords: device, n_brows x 3 FP64, or NULL to keep the rigid-body modes (SCR_SYSTEM only;
 * ignored for MESH_SYSTEM).  Same stream rules as amg_setup; stats.t_setup_ms of the next solve
 * reports this call's time.  Errors: SCR_E_INVALID with the handle unchanged for a different
 * pattern or size, non-finite values or a zero diagonal; an error raised after the values were
 * accepted (a singular block met on a coarse level, SCR_E_OOM, SCR_E_HIP) leaves the handle
 * unusable: every later solve or update on it returns SCR_E_INVALID, destroy it. */
scr_status amg_update(scr_handle* h, const scr_bsr* K, const double* coords, void* stream);

/* Outlet resistance coupling (Sec. 3.5: the consistent linearisation of the reduced outlet models
 * adds alpha_f gamma dt sum_k m_k a_k a_k^T to the velocity block, a_k holding the integrals of
 * N_A n_i over outlet k; for a tangent scaled by 1/(alpha_f gamma dt) the coefficient is m_k).
 * After this call the solves of h use K + sum_k m[k] [a_k; 0][a_k; 0]^T as the outer operator
 * and A + sum_k m[k] a_k a_k^T wherever Algorithms 1 and 2 (and SIMPLE) apply or invert A; the
 * split, S^ and both AMG hierarchies stay those of the sparse K (they are not rebuilt).
 * off: host, n_out + 1 nondecreasing offsets from 0; outlet k owns entries off[k] .. off[k+1]-1.
 * blk: device, off[n_out] block rows (each row at most once over all outlets); a: device,
 * 3 * off[n_out] FP64, the velocity components of a_k at those rows; m: host, n_out FP64.
 * All are copied.  n_out = 0 removes the coupling.  It survives amg_update.  Errors:
 * SCR_E_INVALID (handle kind, offsets, rows out of range or repeated, non-finite values) with
 * the previous coupling kept. */
scr_status scr_set_outlets(scr_handle* h, int n_out, const int64_t* off /* host */, const int32_t* blk,
                           const double* a, const double* m /* host */, void* stream);

/* Solve the corrector system K x = b of Sec. 3.5 (SCR_SYSTEM handle) by right-preconditioned
 * flexible GMRES with the Schur-complement-reduction preconditioner of Sec. 5.2.1 (the inverse of
 * the block LDU factorisation of [A G; D C]), applied by Appendix B, Algorithm 1 (its step 2
 * read as r_p <- r_p - D y^_v), with the Schur action of Algorithm 2 (or, with
 * scr_solve_opts.precond = SCR_PRECOND_SIMPLE, the SIMPLE/SIMPLEC preconditioners of Sec. 5.2.1),
 * to ||b - K x|| <= tol ||b|| (true FP64 residual, checked at exit).
 * b, x: device, 4 * n_brows FP64, node-interleaved [vx vy vz p]; b is not modified; x is
 * caller-allocated and is the initial guess if use_x0, else it is overwritten.  Returns SCR_OK,
 * or SCR_NOT_CONVERGED with x = last iterate; stats (host, may be NULL) are filled either way.
 * Errors: SCR_E_INVALID (NULL pointers, a MESH_SYSTEM handle, options out of range, a handle
 * left unusable by amg_update), SCR_E_BREAKDOWN (non-finite values in a Krylov recurrence),
 * SCR_E_OOM and SCR_E_HIP (workspace allocation on first use, runtime errors). */
scr_status scr_solve(scr_handle* h, const double* b, double* x, const scr_solve_opts* opts /* host */,
                     void* stream, scr_stats* stats /* host */);

/* Solve the mesh-motion system of Sec. 2.2.2 (harmonic extension of the wall displacement into
 * the fluid domain, the same scalar Laplacian L for the x, y and z components; MESH_SYSTEM
 * handle) by CG preconditioned with AMG(L) as in Sec. 5.2.2: L X = B for the three columns at
 * once, each column stopping at ||B_c - L X_c|| <= tol ||B_c||, max_it iterations.  PCG for an
 * FP64 hierarchy, flexible CG (Notay) for an FP32 one or with flexible_cg.
 * b, x: device, n_brows x 3 FP64 interleaved [ux uy uz]; b is not modified; x is overwritten.
 * Returns SCR_OK or SCR_NOT_CONVERGED (stats.mesh_its / mesh_rel per column).  Errors as for
 * scr_solve. */
scr_status mesh_motion_solve(scr_handle* h, const double* b, double* x, const scr_solve_opts* opts /* host */,
                             void* stream, scr_stats* stats /* host */);

/* mesh_motion_solve without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same solve, the
 * same kernels and the bitwise same result, with the CG workspace (15 n + O(1) doubles) in a
 * static device array of 256 MiB that each GPU holds from the first context on it until the
 * process ends, instead of the handle's memory.  Everything else it uses (L, AMG(L), the level
 * vectors, the status slot) was allocated by amg_setup.  Limit: meshes of up to about 2.2M nodes;
 * larger ones return SCR_E_INVALID.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other threads, other streams) race and must be serialised by the caller.
 * Other arguments, results and errors as mesh_motion_solve. */
scr_status mesh_motion_solve_noalloc(scr_handle* h, const double* b, double* x, const scr_solve_opts* opts /* host */,
                                     void* stream, scr_stats* stats /* host */);

scr_status scr_handle_destroy(scr_handle* h);
/* Device memory the handle holds now, and the most it ever held (setup temporaries included);
 * bytes as counted against the context budget. */
int64_t scr_handle_bytes(const scr_handle* h);
int64_t scr_handle_peak_bytes(const scr_handle* h);

/* Device assembly of the corrector tangent matrix K (Sec. 3.5: the consistent linearisation of
 * the semi-discrete unified-continuum equations of Sec. 3.1 (solid, c_m = c_c = 0) and Sec. 3.2
 * (fluid, residual-based VMS), with the first-order generalized-alpha constants of Sec. 3.4,
 * divided by alpha_f gamma dt) on P1 tetrahedra, element integrals by the one-point centroid
 * rule, fluid convection in the Oseen form about a given advective velocity u.  Per element with
 * volume V, local vertices a, b, M_ab = V (1 + delta_ab) / 20, L_ab = V grad N_a . grad N_b,
 * c_t = alpha_m / (alpha_f gamma dt), u_b the centroid velocity and ub.dN = u_b . grad N:
 *   A_ab,ij = delta_ij rho c_t M_ab + visc (delta_ij L_ab + V dN_a,j dN_b,i - 2/3 V dN_a,i dN_b,j)
 *             + tau_C V dN_a,i dN_b,j                                          (fluid only)
 *             + delta_ij [rho V/4 ub.dN_b + tau_M rho^2 ub.dN_a (c_t V/4 + V ub.dN_b)]
 *             + rho M_ab (grad u)_ij                                          (fluid, u given)
 *   G_ab,i  = -V/4 dN_a,i  + tau_M rho V ub.dN_a dN_b,i                      (2nd: fluid, u given)
 *   D_ab,j  =  V/4 dN_b,j  + tau_M rho V dN_a,j ub.dN_b  [+ c_t rho tau_M V/4 dN_a,j]
 *                                             (2nd: fluid, u given; bracket: fluid, vms_dt_coupling)
 *   C_ab    =  tau_M L_ab (fluid),  (c_t / kappa) M_ab (solid)
 * with visc = mu_f (fluid), (alpha_f gamma dt / alpha_m) mu_s (solid), mu_s = E/(2(1+nu)),
 * kappa = E/(3(1-2nu)), and tau_M, tau_C of Sec. 3.2 from the element metric J^-T M J^-1 (M the
 * regular-simplex matrix with 2^(1/3)/2 scaling, C_T = 4, C_I = 36, the u_b.G.u_b term with u).
 * The A and G rows of vertex a go to block row tv[a], its D and C row to tp[a]; the columns of
 * vertex b are tv[b] (A, D) and tp[b] (G, C).  tp differs from tv on the fluid/solid interface,
 * where solid elements take their pressure from a duplicated block row (Sec. 3.3).  Dirichlet
 * dofs (mask) are eliminated: their rows and columns are zeroed and the diagonal set to 1.
 * Every entry is the sum of its element contributions in ascending element order, so the result
 * is bitwise reproducible. */
typedef struct {
    double rho_f, mu_f;         /* fluid density and dynamic viscosity */
    double rho_s, E_s, nu_s;    /* solid density, Young's modulus, Poisson's ratio */
    double dt;                  /* time step */
    double rho_inf;             /* generalized-alpha spectral radius at infinity, in [0, 1] */
    int32_t terms;              /* terms assembled: 1 mass, 2 viscous/elastic, 4 grad-div, 8 G and D,
                                   16 C, 32 convection; 63 = all */
    int32_t vms_dt_coupling;    /* 1: include the bracketed c_t term of D (fluid) */
} scr_tangent_params;

typedef struct scr_assembler scr_assembler;

/* Validate and copy a mesh and a block pattern, and build the per-row incidence lists.
 * tv, tp: device, n_tets x 4 int32 (velocity and pressure block row of each vertex); solid:
 * device, n_tets bytes (nonzero = solid element); row_ptr (n_brows + 1), col_idx: the 4x4 block
 * pattern of K (device; columns strictly ascending per row); coords: device, n_brows x 3 FP64
 * (the coordinates of the velocity rows are used); mask: device, 4 * n_brows bytes (1 = Dirichlet
 * dof).  All are copied.  Errors: SCR_E_INVALID for bad sizes or constants, a malformed pattern,
 * vertex rows out of range, a degenerate element, or an element coupling two rows the pattern
 * does not hold; SCR_E_OOM; SCR_E_HIP. */
scr_status scr_assembler_create(scr_ctx* ctx, int64_t n_tets, const int32_t* tv, const int32_t* tp,
                                const uint8_t* solid, int64_t n_brows, const int32_t* row_ptr,
                                const int32_t* col_idx, const double* coords, const uint8_t* mask,
                                const scr_tangent_params* params /* host */, void* stream,
                                scr_assembler** out /* host */);
/* Assemble K into val (device, 16 * nnzb FP64, 16-byte aligned, row-major 4x4 blocks in the
 * pattern's order; every value is overwritten).  u: device, n_brows x 3 FP64 advective velocity at the velocity rows, or
 * NULL for the tangent at rest (no convection terms; tau without the u.G.u term).  Non-finite u
 * gives non-finite values (amg_setup and amg_update reject them).  Returns after completion. */
scr_status scr_assemble_tangent(scr_assembler* a, const double* u, double* val, void* stream);
int64_t scr_assembler_nnzb(const scr_assembler* a);
int64_t scr_assembler_nbrows(const scr_assembler* a);
/* Release the assembler's device memory.  Every assembly that uses it, on any stream or in a
 * server request, must have finished. */
scr_status scr_assembler_destroy(scr_assembler* a);

/* ---------------------------------------------------------------- time integration
 * The segregated predictor multi-corrector algorithm of Sec. 3.5 with the first-order
 * generalized-alpha method of Sec. 3.4 (same-Y predictor; alpha_m, alpha_f, gamma from the
 * assembler's rho_inf), run on the device for the linear(ised) unified continuum on a fixed mesh:
 * the fluid VMS at rest of Sec. 3.2 (the tangent of scr_assemble_tangent without convection), the
 * small-strain solid of Sec. 3.1 in velocity form with its kinematic equation u_dot = v, the
 * interface pressure duplication of Sec. 3.3, and the mesh motion by harmonic extension of the
 * solid displacement (Sec. 2.2.2; Dirichlet data: the solid displacement on mesh nodes whose
 * velocity row touches a solid element, zero on the other Dirichlet nodes).  The residual of the
 * balance equations is R = K_rate (v_dot - f, p_dot) + K_state (v, p) + K_disp (u_solid, 0) at
 * the intermediate states (f: the body force per unit mass), with the operators the same element
 * integrals give
 * (the corrector tangent divided by alpha_f gamma dt is c_t K_rate + K_state + K_disp / c_t).
 * One step, from the state at t_n:
 *   predictor  y_{n+1} = y_n, y_dot_{n+1} = ((gamma-1)/gamma) y_dot_n (every field);
 *   corrector l = 1, 2, ...: (1-2) du_dot_s = (alpha_f gamma dt/alpha_m) dv_dot_s - R_k/alpha_m,
 *     u_dot_s += du_dot_s, u_s += gamma dt du_dot_s on the solid rows, with dv_dot_s the previous
 *     corrector's velocity-rate increment and R_k = u_dot_s(alpha_m) - v(alpha_f) at the iterate
 *     before that increment was applied (at l = 1: zero and the predictor's R_k);
 *     (3-4) the mesh displacement from mesh_motion_solve and the mesh velocity
 *     v_hat = (u_hat_{n+1} - u_hat_n)/(gamma dt) + ((gamma-1)/gamma) v_hat_n; (7) the residual; (8)
 *     stop when ||R|| <= tol_R ||R_(1)|| or ||R|| <= tol_A; (9) scr_solve of the corrector system
 *     for (dv_dot, dp_dot); (10) v_dot += dv_dot, v += gamma dt dv_dot, p_dot += dp_dot,
 *     p += gamma dt dp_dot.
 * Dirichlet dofs (the assembler's mask) keep zero increments and zero residual.  The reduced
 * outlet models (steps 5-6) and the update of the geometry by the mesh motion are not part of this
 * model.  A step with a new dt re-assembles the operators and re-sets the hierarchies up
 * numerically (amg_update: aggregates and patterns kept). */
typedef struct {
    int32_t max_correctors;    /* l_max, 10 */
    double tol_R;              /* relative stopping tolerance of step 8, 1e-6 */
    double tol_A;              /* absolute stopping tolerance of step 8, 1e-14 */
    double mesh_tol;           /* tolerance of the mesh-motion solves, 1e-10 */
} scr_corrector_opts;

typedef struct {
    int32_t correctors;        /* corrector iterations (the last one only tested the residual) */
    int32_t converged;
    double res0, res;          /* ||R|| at the first corrector and at the last test */
    int64_t linear_its;        /* outer FGMRES iterations over the step's corrector solves */
    int64_t mesh_its;          /* mesh CG iterations (largest column) summed over the correctors */
    int32_t resetups;          /* 1 if the step re-assembled and re-set up for a new dt */
    double t_ms;
} scr_step_stats;

typedef enum {
    SCR_STATE_Y = 0,           /* (v, p): 4 per block row, node-interleaved */
    SCR_STATE_YDOT = 1,        /* (v_dot, p_dot): 4 per block row */
    SCR_STATE_U_SOLID = 2,     /* solid displacement: 3 per block row (zero off solid rows) */
    SCR_STATE_UDOT_SOLID = 3,  /* its rate */
    SCR_STATE_U_MESH = 4,      /* mesh displacement: 3 per mesh node */
    SCR_STATE_V_MESH = 5       /* mesh velocity: 3 per mesh node */
} scr_state_field;

typedef struct scr_stepper scr_stepper;

void scr_default_corrector_opts(scr_corrector_opts* o);   /* o: host */

/* a: the assembler of the system (its pattern, mesh, materials, mask and rho_inf; its dt is
 * replaced by each step's); L: the mesh Laplacian of Sec. 2.2.2 with its Dirichlet nodes eliminated
 * (as for MESH_SYSTEM); L_full: device, nnzb(L) values of the same Laplacian before the elimination
 * (for the lifting of the Dirichlet data); mesh_mask: device, n_L bytes (1 = Dirichlet mesh node);
 * blk_of_phys: device, n_L int32, the velocity block row of each mesh node; solid_rows: device,
 * n_brows bytes (1 = the velocity row touches a solid element); coords: device, n_brows x 3;
 * dt0: the first time step size.  All are copied; the state starts at rest.  The hierarchies are
 * built here (amg_opts, solve_opts for every corrector solve; NULL = defaults). */
scr_status scr_stepper_create(scr_ctx* ctx, scr_assembler* a, const scr_bsr* L, const double* L_full,
                              const uint8_t* mesh_mask, const int32_t* blk_of_phys, const uint8_t* solid_rows,
                              const double* coords, double dt0, const scr_amg_opts* amg /* host */,
                              const scr_solve_opts* solve /* host */, const scr_corrector_opts* copts /* host */,
                              void* stream, scr_stepper** out /* host */);
/* Copy a field of the state at t_n (set = 0: into dst; set = 1: from dst). */
scr_status scr_stepper_state(scr_stepper* s, int field, double* dst, int set, void* stream);
/* One time step of size dt.  f: device, n_brows x 3 body force per unit mass at t_n + alpha_f dt
 * (zero on Dirichlet dofs is not required), or NULL.  Returns SCR_OK, or SCR_NOT_CONVERGED when
 * max_correctors did not meet the stopping test (the state is advanced either way); stats (host,
 * may be NULL).  Errors: SCR_E_INVALID, SCR_E_BREAKDOWN, SCR_E_OOM, SCR_E_HIP, or a failed solve's
 * status. */
scr_status scr_step(scr_stepper* s, double dt, const double* f, void* stream, scr_step_stats* stats /* host */);
scr_status scr_stepper_destroy(scr_stepper* s);

/* Opt-in kernel timing (roofline measurement).  After scr_ctx_profile(ctx, kernel), every launch
 * of that kernel family on handles created from ctx afterwards is bracketed by HIP events on the
 * stream it runs on; scr_ctx_profile_read returns the number of launches, their summed duration
 * (ms) and the summed algorithmic bytes (each matrix and vector byte the kernel must move, once)
 * and resets the counters.  SCR_PROF_SMOOTH_A0: the fused smoother steps (with a matrix
 * product) on level 0 of AMG(A).  Costs two event records per launch; off by default. */
typedef enum { SCR_PROF_OFF = 0, SCR_PROF_SMOOTH_A0 = 1 } scr_prof_kernel;
scr_status scr_ctx_profile(scr_ctx* ctx, int kernel);
scr_status scr_ctx_profile_read(scr_ctx* ctx, int64_t* launches /* host */, double* total_ms /* host */,
                                double* bytes /* host */);

/* Upper bound of the device memory a handle of this size will hold at its peak
 * (scr_handle_peak_bytes: setup temporaries, hierarchies, Krylov workspaces), from a host-side
 * model of the sizes; used for admission control and checked against the measured peak by the
 * tests on the tube workloads. */
int64_t scr_footprint_estimate(int kind, int64_t n_brows, int64_t nnzb, const scr_amg_opts* amg,
                               const scr_solve_opts* solve);

const char* scr_status_str(scr_status s);
const char* scr_last_error(void);

/* ---------------------------------------------------------------- inspection / components
 * Hierarchies: which = 0 AMG(A), 1 AMG(S^), 2 AMG(L).  Fields of a level (copied to host):
 *   0 A.row_ptr (int32, nr+1)   1 A.col_idx (int32, nnzb)   2 A.val (FP64, nnzb*b*b)
 *   3 aggregate of each block row (int32, nr; -1 = isolated); classical: the coarse index of each
 *     C point, -1 on F points
 *   4 P.row_ptr  5 P.col_idx  6 P.val (FP64, b x k blocks)
 *   7 R.row_ptr  8 R.col_idx  9 R.val (FP64, k x b blocks)
 *   10 strong flag per stored block of A (uint8)   11 dead coarse dof flags (uint8, nagg*k)
 *   12 D^-1 blocks (FP64, nr*b*b)   13 near-null space B (FP64, nr*b x k)
 *   15 classical: the function of each scalar row (uint8, nr)
 * info = [nr, b, k, nnzb(A), nagg, nnzb(P), nnzb(R), n_coarsest]; lam = lambda_hat.  Classical
 * hierarchies are scalar (b = k = 1, level 0 the scalar rows of the blocks); nagg = C points. */
scr_status scr_hier_levels(scr_handle* h, int which, int* nlev /* host */);
scr_status scr_hier_level_info(scr_handle* h, int which, int level, int64_t* info /* host, 8 */,
                               double* lam /* host */);
scr_status scr_hier_level_copy(scr_handle* h, int which, int level, int field, void* dst /* host */);

/* Split matrices of an SCR handle: which 0 A, 1 G, 2 D, 3 C, 4 S^; field 0 row_ptr, 1 col_idx,
 * 2 values (FP64); info (host, 4) = [nr, nnzb, br, bc] is always filled. */
scr_status scr_matrix_copy(scr_handle* h, int which, int field, void* dst /* host, may be NULL */,
                           int64_t* info /* host */);

/* Component operators on split vectors (velocity part 3n node-interleaved, then pressure n):
 *   0 y = K x (4n -> 4n)          1 y = A x (3n)              2 y = V-cycle of AMG(A) (3n)
 *   3 y = V-cycle of AMG(S^) (n)  4 y = S x by Algorithm 2 (n) 5 y = P_SCR^-1 x, Algorithm 1 (4n)
 *   6 y = G x (n -> 3n)           7 y = D x (3n -> n)          8 y = C x (n)
 *   9 y = S^ x (n)               10 y = L x (mesh handle, n)  11 y = V-cycle of AMG(L) (n)
 *  12 y = P_SIMPLE^-1 x (4n)     13 y = d, the diagonal used in S^ (3n; x unused)
 * x, y: device FP64. */
scr_status scr_apply(scr_handle* h, int op, const double* x, double* y, const scr_solve_opts* opts,
                     void* stream);

/* ---------------------------------------------------------------- serving
 * A server keeps a FIFO queue of solve requests and max_slots worker threads, each with its own
 * HIP stream.  A request is admitted when a slot is free and the sum of the footprint estimates
 * (scr_footprint_estimate) of the admitted requests stays within hbm_budget (0 = the context's
 * budget, or unlimited); requests that arrive while others run are admitted as slots and memory
 * free up, and their kernels overlap on the device.  A request whose footprint alone exceeds the
 * budget is rejected (SCR_E_OOM), never queued forever.  Each request builds its hierarchies
 * once (amg_setup) and reuses them for its n_rhs successive corrections (the multi-corrector
 * loop of Sec. 3.5), and for its mesh-motion solves when L is given.  The tangent is frozen
 * unless the request gives new values for a correction, or a new advective velocity with an
 * assembler (the tangent is then assembled on the device): the hierarchies are re-set up
 * numerically (amg_update) before that correction's solve.
 * All device arrays of a request are borrowed until srv_wait/srv_poll reports it done. */
typedef struct scr_server scr_server;

typedef struct {
    scr_bsr K;                     /* SCR_SYSTEM matrix (device arrays) */
    const double* coords;          /* device, n_brows x 3 */
    int n_rhs;                     /* successive corrections, 1..64 */
    const double* const* b;        /* host array of n_rhs device pointers (4 n_brows each) */
    double* const* x;              /* host array of n_rhs device pointers (outputs) */
    const scr_bsr* L;              /* optional mesh Laplacian (NULL = none) */
    const double* const* bm;       /* n_rhs device pointers (n_L x 3 each), if L */
    double* const* xm;             /* n_rhs device pointers (outputs), if L */
    const double* const* vals;     /* NULL (frozen tangent), or n_rhs device pointers: vals[c]
                                      (c >= 1; NULL keeps the previous values) are the K values of
                                      correction c on K's pattern (nnzb * 16 each); vals[0] is
                                      ignored (K.val is the first correction's matrix) */
    scr_assembler* tangent;        /* NULL, or an assembler created on K's pattern (same n_brows and
                                      nnzb): the tangents are then assembled on the device at the
                                      advective velocities u, and vals is not read.  The first
                                      correction's matrix is the tangent at u[0] (NULL = at rest)
                                      and K.val is not read; for c >= 1 a non-NULL u[c] gives a new
                                      tangent, assembled and re-set up numerically before that
                                      correction's solve (NULL keeps the previous one).  The values
                                      live in a buffer of 16 nnzb FP64 that the request holds while
                                      it runs (counted in its footprint).  One assembler may serve
                                      requests that run concurrently. */
    const double* const* u;        /* n_rhs device pointers (n_brows x 3 each, or NULL), if tangent */
} scr_request;

typedef struct {
    scr_status status;             /* worst status over the request's solves */
    int64_t n_solves;
    double latency_ms;             /* submit -> last correction done */
    double queue_ms;               /* submit -> admission */
    double setup_ms, solve_ms;     /* summed over the request (setup_ms includes re-setups) */
    int64_t footprint;             /* admission estimate (bytes) */
    int64_t device_bytes;          /* measured peak of the request's handle(s) */
    scr_stats last;                /* stats of the last SCR solve */
} srv_result;

scr_status srv_create(scr_ctx* ctx, int max_slots, int64_t hbm_budget, const scr_amg_opts* amg /* host */,
                      const scr_solve_opts* solve /* host */, scr_server** out /* host */);
/* Non-blocking; the request struct and its pointer arrays are copied. */
scr_status srv_submit(scr_server* s, const scr_request* r /* host */, int64_t* id /* host */);
/* done = 1 when the request has finished (result filled), 0 otherwise.  Non-blocking. */
scr_status srv_poll(scr_server* s, int64_t id, int* done /* host */, srv_result* res /* host */);
/* Block until the request has finished. */
scr_status srv_wait(scr_server* s, int64_t id, srv_result* res /* host */);
/* Block until every submitted request has finished; max_active (host, may be NULL) receives the
 * largest number of requests that ran at the same time. */
scr_status srv_drain(scr_server* s, int* max_active);
void srv_destroy(scr_server* s);

#ifdef __cplusplus
}
#endif
#endif
