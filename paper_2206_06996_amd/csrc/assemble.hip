// assemble.hip -- device assembly of the corrector tangent matrix on P1 tetrahedra (Sec. 3.1,
// 3.2 and 3.5: the linearised unified-continuum VMS tangent, divided by alpha_f gamma dt) into a
// fixed 4x4 block pattern.
//
// One thread per stored 4x4 block.  Each block row keeps its incident (element, local vertex)
// pairs sorted by element, so every entry is the sum of its element contributions in ascending
// element order: the result does not depend on scheduling (no atomics in the value pass).  A
// thread recomputes the geometry, tau and the advective quantities of each element that couples
// its row and column (an element is seen by the 16 blocks of its vertex pairs, more on the
// fluid/solid interface); the values are accumulated in registers and written once.
#include <climits>
#include <cmath>
#include <memory>

#include "common.h"
#include "kernels.h"

struct scr_assembler {
    scr::Ctx* ctx = nullptr;
    std::unique_ptr<scr::Arena> ar;
    int64_t n_tets = 0, nb = 0, nnzb = 0, n_inc = 0;
    int32_t *tv = nullptr, *tp = nullptr, *rp = nullptr, *ci = nullptr, *inc_off = nullptr;
    int64_t* inc = nullptr;       // per block row, sorted: ((4 e + a) << 2) | role
    int32_t* rowof = nullptr;     // block row of each stored block
    uint8_t *solid = nullptr, *mask = nullptr;
    double* xyz = nullptr;
    scr_tangent_params p{};
};

namespace scr {
namespace {

// constants of one assembly (Sec. 3.4: first-order generalized-alpha; Sec. 3.1: solid moduli) and
// the coefficient of each term in the assembled form (FORM_TANGENT: the corrector tangent divided
// by alpha_f gamma dt; the other forms are the parts of the linear(ised) semi-discrete residual that
// act on the rates, on the state and on the solid displacement, see OperatorForm)
struct TanPrm {
    double rho_f, mu_f, rho_s, ct, visc_s, kappa, dt;
    int terms, dtc;
    double c_mass;          // times rho M (both media)
    double c_visc_f;        // fluid viscous coefficient (mu_f or 0)
    double c_visc_s;        // solid elastic coefficient
    double c_gd;            // times tau_C grad-div (fluid)
    double c_gdiv;          // G and D (1 or 0)
    double c_dtc;           // the fine-scale rate term of D (fluid, with vms_dt_coupling)
    double c_cf;            // times tau_M L (fluid pressure block)
    double c_cs;            // times M (solid pressure block)
    int conv;               // Oseen convection terms allowed
    int unit_diag;          // Dirichlet dofs: unit diagonal (the tangent) or zero rows (residual parts)
};

TanPrm tan_prm(const scr_tangent_params& p, int form = FORM_TANGENT) {
    const double am = 0.5 * (3.0 - p.rho_inf) / (1.0 + p.rho_inf);
    const double af = 1.0 / (1.0 + p.rho_inf), g = 1.0 / (1.0 + p.rho_inf);
    TanPrm t;
    t.rho_f = p.rho_f; t.mu_f = p.mu_f; t.rho_s = p.rho_s; t.dt = p.dt;
    t.ct = am / (af * g * p.dt);
    const double mu_s = p.E_s / (2.0 * (1.0 + p.nu_s));
    t.visc_s = (af * g * p.dt / am) * mu_s;
    t.kappa = p.E_s / (3.0 * (1.0 - 2.0 * p.nu_s));
    t.terms = p.terms;
    t.dtc = p.vms_dt_coupling;
    t.c_mass = t.c_visc_f = t.c_visc_s = t.c_gd = t.c_gdiv = t.c_dtc = t.c_cf = t.c_cs = 0.0;
    t.conv = 0;
    t.unit_diag = 0;
    switch (form) {
        case FORM_TANGENT:
            t.c_mass = t.ct; t.c_visc_f = t.mu_f; t.c_visc_s = t.visc_s; t.c_gd = 1.0; t.c_gdiv = 1.0;
            t.c_dtc = t.ct; t.c_cf = 1.0; t.c_cs = t.ct / t.kappa; t.conv = 1; t.unit_diag = 1;
            break;
        case FORM_RATE:       // acts on (v_dot, p_dot): rho M, the solid pressure mass M / kappa
            t.c_mass = 1.0; t.c_dtc = 1.0; t.c_cs = 1.0 / t.kappa;
            break;
        case FORM_STATE:      // acts on (v, p): fluid viscous and grad-div, G and D, tau_M L
            t.c_visc_f = t.mu_f; t.c_gd = 1.0; t.c_gdiv = 1.0; t.c_cf = 1.0;
            break;
        case FORM_DISP:       // acts on the solid displacement: the deviatoric elastic stiffness
            t.c_visc_s = mu_s;
            break;
        default: throw Error(SCR_E_INVALID, "unknown operator form");
    }
    return t;
}

// Shape-function gradients of a tetrahedron: with the edge vectors e_k = x_k - x_0 (k = 1..3) and
// det = e_1 . (e_2 x e_3), grad N_1 = (e_2 x e_3)/det, grad N_2 = (e_3 x e_1)/det,
// grad N_3 = (e_1 x e_2)/det (the rows of the inverse Jacobian), grad N_0 = -(sum of the others).
// Returns det (six times the signed volume).
__device__ __forceinline__ double tet_shape(const double (&x)[4][3], double (&dN)[4][3]) {
    double e[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) e[k][i] = x[k + 1][i] - x[0][i];
    double c[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double* u = e[(k + 1) % 3];
        const double* w = e[(k + 2) % 3];
        c[k][0] = u[1] * w[2] - u[2] * w[1];
        c[k][1] = u[2] * w[0] - u[0] * w[2];
        c[k][2] = u[0] * w[1] - u[1] * w[0];
    }
    const double det = e[0][0] * c[0][0] + e[0][1] * c[0][1] + e[0][2] * c[0][2];
    const double inv = 1.0 / det;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        dN[1][i] = c[0][i] * inv;
        dN[2][i] = c[1][i] * inv;
        dN[3][i] = c[2][i] * inv;
        dN[0][i] = -(dN[1][i] + dN[2][i] + dN[3][i]);
    }
    return det;
}

// tau_M and tau_C of the fluid VMS (Sec. 3.2) from the element metric G = J^-T M J^-1, M the
// regular-simplex matrix (2^(1/3)/2 times [2 1 1; 1 2 1; 1 1 2]), C_T = 4, C_I = 36; ub is the
// advective velocity at the centroid (zero at rest).
__device__ __forceinline__ void fluid_tau(const double (&dN)[4][3], const double (&ub)[3], const TanPrm& P,
                                          double& tauM, double& tauC) {
    const double c = 0.6299605249474366;   // 2^(1/3) / 2
    double G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // sum_kl dN_k,i M_kl dN_l,j with M = c (I + 1 1^T)
            const double s1 = dN[1][i] + dN[2][i] + dN[3][i];
            const double s2 = dN[1][j] + dN[2][j] + dN[3][j];
            G[i][j] = c * (dN[1][i] * dN[1][j] + dN[2][i] * dN[2][j] + dN[3][i] * dN[3][j] + s1 * s2);
        }
    double GG = 0.0, trG = 0.0, uGu = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        trG += G[i][i];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            GG += G[i][j] * G[i][j];
            uGu += ub[i] * G[i][j] * ub[j];
        }
    }
    const double nu = P.mu_f / P.rho_f;
    tauM = 1.0 / (P.rho_f * sqrt(4.0 / (P.dt * P.dt) + uGu + 36.0 * nu * nu * GG));
    tauC = 1.0 / (tauM * trG);
}

// position of column c in the sorted columns ci[lo, hi), or -1
__device__ __forceinline__ int32_t find_col(const int32_t* __restrict__ ci, int32_t lo, int32_t hi, int32_t c) {
    int32_t a = lo, b = hi;
    while (a < b) {
        const int32_t m = (a + b) >> 1;
        if (ci[m] < c) a = m + 1;
        else b = m;
    }
    return (a < hi && ci[a] == c) ? a : -1;
}

// ---------------------------------------------------------------- set-up kernels
// rows whose pattern is malformed: columns out of range or not strictly ascending
__global__ void pattern_check_k(int64_t nb, int64_t nnzb, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ ci, int* __restrict__ err) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int32_t lo = rp[r], hi = rp[r + 1];
    bool bad = lo < 0 || hi < lo || hi > nnzb;
    for (int32_t q = lo; q < hi && !bad; ++q) bad = ci[q] < 0 || ci[q] >= nb || (q > lo && ci[q] <= ci[q - 1]);
    if (bad) atomicOr(err, 1);
}

// per element: vertex rows in range, a nondegenerate finite geometry, and every block position the
// element writes present in the pattern
__global__ void element_check_k(int64_t nt, int64_t nb, const int32_t* __restrict__ tv, const int32_t* __restrict__ tp,
                                const double* __restrict__ xyz, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ ci, int* __restrict__ err) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nt) return;
    int32_t va[4], pa[4];
    for (int a = 0; a < 4; ++a) {
        va[a] = tv[4 * e + a];
        pa[a] = tp[4 * e + a];
        if (va[a] < 0 || va[a] >= nb || pa[a] < 0 || pa[a] >= nb) {
            atomicOr(err, 2);
            return;
        }
    }
    double x[4][3], dN[4][3];
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) x[a][i] = xyz[3 * (int64_t)va[a] + i];
    const double det = tet_shape(x, dN);
    if (!(det != 0.0) || !isfinite(det)) atomicOr(err, 4);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const int32_t rows[2] = {va[a], pa[a]}, cols[2] = {va[b], pa[b]};
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t)
                    if (find_col(ci, rp[rows[s]], rp[rows[s] + 1], cols[t]) < 0) atomicOr(err, 8);
        }
}

// incidence: element vertex (e, a) touches block row tv (velocity rows, role 1) and tp (pressure
// row, role 2); they coincide (role 3) off the fluid/solid interface
__global__ void inc_count_k(int64_t n4, const int32_t* __restrict__ tv, const int32_t* __restrict__ tp,
                            int32_t* __restrict__ cnt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const int32_t v = tv[t], p = tp[t];
    atomicAdd(&cnt[v], 1);
    if (p != v) atomicAdd(&cnt[p], 1);
}
__global__ void inc_fill_k(int64_t n4, const int32_t* __restrict__ tv, const int32_t* __restrict__ tp,
                           int32_t* __restrict__ cur, int64_t* __restrict__ inc) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const int32_t v = tv[t], p = tp[t];
    if (p == v) {
        inc[atomicAdd(&cur[v], 1)] = (t << 2) | 3;
    } else {
        inc[atomicAdd(&cur[v], 1)] = (t << 2) | 1;
        inc[atomicAdd(&cur[p], 1)] = (t << 2) | 2;
    }
}
// each row's list in ascending key order (= element order): insertion sort, the lists are short
__global__ void inc_sort_k(int64_t nb, const int32_t* __restrict__ off, int64_t* __restrict__ inc) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int32_t lo = off[r], hi = off[r + 1];
    for (int32_t i = lo + 1; i < hi; ++i) {
        const int64_t k = inc[i];
        int32_t j = i - 1;
        while (j >= lo && inc[j] > k) {
            inc[j + 1] = inc[j];
            --j;
        }
        inc[j + 1] = k;
    }
}

// ---------------------------------------------------------------- the tangent
// Element rows of local vertex a, per column vertex b (entries (i, j), i, j = 0..2 velocity, 3
// pressure; V the volume, M_ab = V (1 + delta_ab)/20 the P1 mass, L_ab = V grad N_a . grad N_b):
//   A_ij = delta_ij rho c_t M_ab                                                  (mass, bit 1)
//        + visc (delta_ij L_ab + V dN_a,j dN_b,i - 2/3 V dN_a,i dN_b,j)          (bit 2)
//        + tau_C V dN_a,i dN_b,j                          (fluid grad-div stabilisation, bit 4)
//        + delta_ij [rho (V/4) ub.dN_b + tau_M rho^2 (ub.dN_a)(c_t V/4 + V ub.dN_b)]
//        + rho M_ab grad u_ij                           (fluid convection, Oseen form, bit 32)
//   G_i  = -(V/4) dN_a,i  [+ tau_M rho V (ub.dN_a) dN_b,i]                        (bit 8 [32])
//   D_j  =  (V/4) dN_b,j  [+ c_t rho tau_M (V/4) dN_a,j]  [+ tau_M rho V dN_a,j (ub.dN_b)]
//   C    =  tau_M L_ab (fluid),  (c_t/kappa) M_ab (solid)                          (bit 16)
// visc = mu_f for fluid, (alpha_f gamma dt/alpha_m) mu_s for solid.  The A and G rows go to block
// row tv[a] (role 1), the D and C row to tp[a] (role 2); columns tv[b] (A, D) and tp[b] (G, C).
// One thread per stored block (r, c): it walks row r's incidence list (ascending elements), skips
// the elements that do not hold c as a velocity or pressure column, and accumulates the 16 entries
// of the block in registers; each block is written once (consecutive threads write consecutive
// blocks), then the Dirichlet elimination is applied to it.
__global__ void __launch_bounds__(256) tangent_blocks_k(int64_t nnzb, const int32_t* __restrict__ rowof,
                                                        const int32_t* __restrict__ ci, const int32_t* __restrict__ ioff,
                                                        const int64_t* __restrict__ inc, const int32_t* __restrict__ tv,
                                                        const int32_t* __restrict__ tp, const uint8_t* __restrict__ solid,
                                                        const double* __restrict__ xyz, const double* __restrict__ u,
                                                        const uint8_t* __restrict__ mask, TanPrm P,
                                                        double* __restrict__ val) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnzb) return;
    const int32_t r = rowof[q], c = ci[q];
    double acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.0;
    const bool t_mass = P.terms & 1, t_visc = P.terms & 2, t_gd = P.terms & 4, t_gdiv = (P.terms & 8) && P.c_gdiv != 0.0,
               t_c = P.terms & 16;
    for (int32_t k = ioff[r]; k < ioff[r + 1]; ++k) {
        const int64_t key = inc[k];
        const int64_t e = key >> 4;
        const int a = (int)((key >> 2) & 3);
        const int role = (int)(key & 3);
        typedef int I4 __attribute__((ext_vector_type(4)));
        const I4 va = *reinterpret_cast<const I4*>(tv + 4 * e);
        const I4 pa = *reinterpret_cast<const I4*>(tp + 4 * e);
        // the column vertex b of c (velocity and pressure columns; at most one b each)
        int bv = -1, bq = -1;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (va[b] == c) bv = b;
            if (pa[b] == c) bq = b;
        }
        if (bv < 0 && bq < 0) continue;
        double x[4][3];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 3; ++i) x[b][i] = xyz[3 * (int64_t)va[b] + i];
        double dN[4][3];
        const double V = fabs(tet_shape(x, dN)) / 6.0;
        const bool sol = solid[e] != 0;
        const bool conv = !sol && u != nullptr && (P.terms & 32) && P.conv;
        double ub[3] = {0.0, 0.0, 0.0}, gu[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        if (conv) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double ui = u[3 * (int64_t)va[b] + i];
                    ub[i] += 0.25 * ui;
#pragma unroll
                    for (int j = 0; j < 3; ++j) gu[i][j] += ui * dN[b][j];
                }
        }
        double tauM = 0.0, tauC = 0.0, rho, visc;
        if (!sol) {
            fluid_tau(dN, ub, P, tauM, tauC);
            rho = P.rho_f;
            visc = P.c_visc_f;
        } else {
            rho = P.rho_s;
            visc = P.c_visc_s;
        }
        const double gd = sol ? 0.0 : P.c_gd * tauC;
        double dNa[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) dNa[i] = a == 0 ? dN[0][i] : a == 1 ? dN[1][i] : a == 2 ? dN[2][i] : dN[3][i];
        const double ua = ub[0] * dNa[0] + ub[1] * dNa[1] + ub[2] * dNa[2];
        if (bv >= 0) {
            double dNb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dNb[i] = bv == 0 ? dN[0][i] : bv == 1 ? dN[1][i] : bv == 2 ? dN[2][i] : dN[3][i];
            const double Mab = V * (a == bv ? 2.0 : 1.0) / 20.0;
            const double Lab = V * (dNa[0] * dNb[0] + dNa[1] * dNb[1] + dNa[2] * dNb[2]);
            const double uB = ub[0] * dNb[0] + ub[1] * dNb[1] + ub[2] * dNb[2];
            if (role & 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        double v = 0.0;
                        if (t_mass && i == j) v += rho * P.c_mass * Mab;
                        if (t_visc)
                            v += visc * ((i == j ? Lab : 0.0) + V * dNa[j] * dNb[i] - (2.0 / 3.0) * V * dNa[i] * dNb[j]);
                        if (t_gd) v += gd * V * dNa[i] * dNb[j];
                        if (conv) {
                            if (i == j) v += rho * (V / 4.0) * uB + tauM * rho * rho * ua * (P.ct * (V / 4.0) + V * uB);
                            v += rho * Mab * gu[i][j];
                        }
                        acc[4 * i + j] += v;
                    }
            }
            if (role & 2) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double d = 0.0;
                    if (P.terms & 8) {
                        if (t_gdiv) d = (V / 4.0) * dNb[j];
                        if (!sol && P.dtc) d += P.c_dtc * rho * tauM * (V / 4.0) * dNa[j];
                    }
                    if (conv) d += tauM * rho * V * dNa[j] * uB;
                    acc[12 + j] += d;
                }
            }
        }
        if (bq >= 0) {
            double dNb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dNb[i] = bq == 0 ? dN[0][i] : bq == 1 ? dN[1][i] : bq == 2 ? dN[2][i] : dN[3][i];
            if (role & 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double g = t_gdiv ? -(V / 4.0) * dNa[i] : 0.0;
                    if (conv) g += tauM * rho * V * ua * dNb[i];
                    acc[4 * i + 3] += g;
                }
            }
            if ((role & 2) && t_c) {
                const double Mab = V * (a == bq ? 2.0 : 1.0) / 20.0;
                const double Lab = V * (dNa[0] * dNb[0] + dNa[1] * dNb[1] + dNa[2] * dNb[2]);
                acc[15] += sol ? P.c_cs * Mab : P.c_cf * tauM * Lab;
            }
        }
    }
    // Dirichlet elimination: rows and columns of constrained dofs zeroed, unit diagonal
    typedef double D2 __attribute__((ext_vector_type(2)));
    D2* out = reinterpret_cast<D2*>(val + 16 * q);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint8_t mr = mask[4 * (int64_t)r + i];
        double w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint8_t mc = mask[4 * (int64_t)c + j];
            w[j] = (mr || mc) ? ((c == r && i == j && P.unit_diag) ? 1.0 : 0.0) : acc[4 * i + j];
        }
        out[2 * i] = D2{w[0], w[1]};
        out[2 * i + 1] = D2{w[2], w[3]};
    }
}

// block row of every stored block
__global__ void row_of_k(int64_t nb, const int32_t* __restrict__ rp, int32_t* __restrict__ rowof) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) rowof[q] = (int32_t)r;
}

scr_status asm_fail(const std::exception& e) { return status_of(e); }

}  // namespace
}  // namespace scr

using namespace scr;

scr_status scr_assembler_create(scr_ctx* ctx, int64_t n_tets, const int32_t* tv, const int32_t* tp,
                                const uint8_t* solid, int64_t n_brows, const int32_t* row_ptr,
                                const int32_t* col_idx, const double* coords, const uint8_t* mask,
                                const scr_tangent_params* params, void* stream, scr_assembler** out) {
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<scr_assembler> A;
    try {
        if (!ctx || !out || !params) throw Error(SCR_E_INVALID, "NULL ctx, out or params");
        *out = nullptr;
        if (n_tets < 1 || n_brows < 1) throw Error(SCR_E_INVALID, "n_tets and n_brows must be positive");
        if (!tv || !tp || !solid || !row_ptr || !col_idx || !coords || !mask)
            throw Error(SCR_E_INVALID, "NULL input array");
        if (8 * n_tets > INT32_MAX) throw Error(SCR_E_INVALID, "too many elements (the incidence lists use 32-bit offsets)");
        const scr_tangent_params& p = *params;
        for (double v : {p.rho_f, p.mu_f, p.rho_s, p.E_s, p.dt})
            if (!(v > 0.0) || !std::isfinite(v)) throw Error(SCR_E_INVALID, "physical constants must be positive");
        if (!(p.nu_s > -1.0 && p.nu_s < 0.5)) throw Error(SCR_E_INVALID, "nu_s must lie in (-1, 0.5)");
        if (!(p.rho_inf >= 0.0 && p.rho_inf <= 1.0)) throw Error(SCR_E_INVALID, "rho_inf must lie in [0, 1]");
        if (p.terms < 0 || p.terms > 63) throw Error(SCR_E_INVALID, "terms must be a mask of bits 1..32");
        HIPCHK(hipSetDevice(ctx->c.device));
        A.reset(new scr_assembler());
        A->ctx = &ctx->c;
        A->ar.reset(new Arena(&ctx->c, s));
        Arena& ar = *A->ar;
        A->n_tets = n_tets;
        A->nb = n_brows;
        A->p = p;
        int32_t ends[2];
        HIPCHK(hipMemcpyAsync(&ends[0], row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&ends[1], row_ptr + n_brows, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (ends[0] != 0 || ends[1] < n_brows) throw Error(SCR_E_INVALID, "row_ptr must start at 0 and cover the diagonal");
        A->nnzb = ends[1];
        A->tv = ar.make<int32_t>(4 * n_tets);
        A->tp = ar.make<int32_t>(4 * n_tets);
        A->solid = ar.make<uint8_t>(n_tets);
        A->rp = ar.make<int32_t>(n_brows + 1);
        A->ci = ar.make<int32_t>(A->nnzb);
        A->xyz = ar.make<double>(3 * n_brows);
        A->mask = ar.make<uint8_t>(4 * n_brows);
        copy_dev(A->tv, tv, 4 * n_tets * sizeof(int32_t), s);
        copy_dev(A->tp, tp, 4 * n_tets * sizeof(int32_t), s);
        copy_dev(A->solid, solid, n_tets, s);
        copy_dev(A->rp, row_ptr, (n_brows + 1) * sizeof(int32_t), s);
        copy_dev(A->ci, col_idx, A->nnzb * sizeof(int32_t), s);
        copy_dev(A->xyz, coords, 3 * n_brows * sizeof(double), s);
        copy_dev(A->mask, mask, 4 * n_brows, s);
        int* err = ar.make<int>(1);
        zero_dev(err, sizeof(int), s);
        pattern_check_k<<<cdiv(n_brows, 256), 256, 0, s>>>(n_brows, A->nnzb, A->rp, A->ci, err);
        check_launch("pattern_check");
        int herr = 0;
        HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (herr) throw Error(SCR_E_INVALID, "malformed pattern (row_ptr decreasing, columns out of range or unsorted)");
        element_check_k<<<cdiv(n_tets, 256), 256, 0, s>>>(n_tets, n_brows, A->tv, A->tp, A->xyz, A->rp, A->ci, err);
        check_launch("element_check");
        HIPCHK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (herr & 2) throw Error(SCR_E_INVALID, "element vertex row out of range");
        if (herr & 4) throw Error(SCR_E_INVALID, "degenerate or non-finite element");
        if (herr & 8) throw Error(SCR_E_INVALID, "an element couples two block rows the pattern does not hold");
        // incidence lists
        int32_t* cnt = ar.make<int32_t>(n_brows);
        zero_dev(cnt, n_brows * sizeof(int32_t), s);
        inc_count_k<<<cdiv(4 * n_tets, 256), 256, 0, s>>>(4 * n_tets, A->tv, A->tp, cnt);
        check_launch("inc_count");
        A->inc_off = ar.make<int32_t>(n_brows + 1);
        A->n_inc = scan_i32(cnt, A->inc_off, n_brows, ar, s);
        A->inc = ar.make<int64_t>(A->n_inc);
        copy_dev(cnt, A->inc_off, n_brows * sizeof(int32_t), s);
        inc_fill_k<<<cdiv(4 * n_tets, 256), 256, 0, s>>>(4 * n_tets, A->tv, A->tp, cnt, A->inc);
        check_launch("inc_fill");
        inc_sort_k<<<cdiv(n_brows, 256), 256, 0, s>>>(n_brows, A->inc_off, A->inc);
        check_launch("inc_sort");
        A->rowof = ar.make<int32_t>(A->nnzb);
        row_of_k<<<cdiv(n_brows, 256), 256, 0, s>>>(n_brows, A->rp, A->rowof);
        check_launch("row_of");
        ar.free(cnt);
        ar.free(err);
        HIPCHK(hipStreamSynchronize(s));
        *out = A.release();
        return SCR_OK;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        return asm_fail(e);
    }
}

namespace scr {
void assemble_form(scr_assembler* A, int form, double dt, const double* u, double* val, hipStream_t s) {
    if (!A || !val) throw Error(SCR_E_INVALID, "NULL assembler or val");
    if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(SCR_E_INVALID, "dt must be positive");
    if (reinterpret_cast<uintptr_t>(val) % 16 != 0) throw Error(SCR_E_INVALID, "val must be 16-byte aligned");
    scr_tangent_params p = A->p;
    p.dt = dt;
    const TanPrm P = tan_prm(p, form);
    tangent_blocks_k<<<cdiv(A->nnzb, 256), 256, 0, s>>>(A->nnzb, A->rowof, A->ci, A->inc_off, A->inc, A->tv, A->tp,
                                                         A->solid, A->xyz, form == FORM_TANGENT ? u : nullptr,
                                                         A->mask, P, val);
    check_launch("tangent_blocks");
}
double asmb_rho_inf(const scr_assembler* A) { return A->p.rho_inf; }
void asmb_pattern(const scr_assembler* A, int32_t* rp, int32_t* ci, hipStream_t s) {
    copy_dev(rp, A->rp, (A->nb + 1) * sizeof(int32_t), s);
    copy_dev(ci, A->ci, A->nnzb * sizeof(int32_t), s);
}
}  // namespace scr

scr_status scr_assemble_tangent(scr_assembler* A, const double* u, double* val, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!A || !val) throw Error(SCR_E_INVALID, "NULL assembler or val");
        if (reinterpret_cast<uintptr_t>(val) % 16 != 0) throw Error(SCR_E_INVALID, "val must be 16-byte aligned");
        HIPCHK(hipSetDevice(A->ctx->device));
        tangent_blocks_k<<<cdiv(A->nnzb, 256), 256, 0, s>>>(A->nnzb, A->rowof, A->ci, A->inc_off, A->inc, A->tv, A->tp,
                                                             A->solid, A->xyz, u, A->mask, tan_prm(A->p), val);
        check_launch("tangent_blocks");
        HIPCHK(hipStreamSynchronize(s));
        return SCR_OK;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        return asm_fail(e);
    }
}

int64_t scr_assembler_nnzb(const scr_assembler* A) { return A ? A->nnzb : 0; }
int64_t scr_assembler_nbrows(const scr_assembler* A) { return A ? A->nb : 0; }

scr_status scr_assembler_destroy(scr_assembler* A) {
    if (!A) return SCR_OK;
    delete A;   // the arena synchronises its stream and returns every block to the context cache
    return SCR_OK;
}
