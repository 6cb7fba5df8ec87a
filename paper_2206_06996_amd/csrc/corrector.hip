// corrector.hip -- time integration by the segregated predictor multi-corrector algorithm of
// Sec. 3.5 with the first-order generalized-alpha method of Sec. 3.4, on the device, for the
// linear(ised) unified continuum on a fixed mesh: the fluid VMS at rest (Sec. 3.2), the
// small-strain solid in velocity form with its kinematic equation u_dot = v (Sec. 3.1, c_m = c_c =
// 0), the interface pressure duplication (Sec. 3.3) and the mesh motion by harmonic extension
// with the solid displacement as its Dirichlet data (Sec. 2.2.2, the unified viewpoint of the
// remark closing Sec. 3.5).  Every corrector assembles the residual of the balance equations at
// the intermediate states on the device, tests it, and solves the 2x2 block corrector system with
// scr_solve; the solid displacement, the mesh displacement and velocity, and the velocity and
// pressure are updated by device kernels.  A new time step size re-assembles the operators and
// re-sets the hierarchies up numerically (amg_update) on the same patterns.
#include <chrono>
#include <cmath>
#include <memory>

#include "solver.h"

using namespace scr;

struct scr_stepper {
    scr_ctx* sctx = nullptr;
    Ctx* ctx = nullptr;
    std::unique_ptr<Arena> ar;
    scr_assembler* asmb = nullptr;
    int64_t nb = 0, nnzb = 0, nL = 0;
    double dt = 0.0, am = 0.0, af = 0.0, gam = 0.0;
    scr_corrector_opts co{};
    scr_solve_opts so{};
    scr_amg_opts ao{};
    int32_t *rp = nullptr, *ci = nullptr, *blk_of_phys = nullptr;
    uint8_t *solid_rows = nullptr, *mesh_mask = nullptr;
    double *Kt = nullptr, *Kr = nullptr, *Ks = nullptr, *Kd = nullptr, *coords = nullptr;
    DSell<double> Lfull;
    scr_handle *h = nullptr, *hm = nullptr;
    const int32_t *Lrp = nullptr, *Lci = nullptr;
    // state at t_n and the iterate at t_{n+1}: y = (v, p) and its rate (4 per block row); the solid
    // displacement and its rate (3 per velocity row); the mesh displacement and velocity (3 per node)
    double *yn = nullptr, *y1 = nullptr, *ydn = nullptr, *yd1 = nullptr;
    double *usn = nullptr, *us1 = nullptr, *usdn = nullptr, *usd1 = nullptr;
    double *mun = nullptr, *mu1 = nullptr, *mvn = nullptr, *mv1 = nullptr;
    // work vectors
    double *yaf = nullptr, *ydam = nullptr, *uaf = nullptr, *R = nullptr, *Rk = nullptr, *rhs = nullptr,
           *dyd = nullptr, *dvd = nullptr, *uD = nullptr, *lift = nullptr, *bm = nullptr;
    Reducer red;
    StatusSlot slot;
};

namespace {

// x1 = xn;  xd1 = c xd_n   (the same-Y predictor, c = (gamma - 1) / gamma)
__global__ void predictor_k(int64_t n, const double* __restrict__ xn, const double* __restrict__ xdn,
                            double* __restrict__ x1, double* __restrict__ xd1, double c) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x1[i] = xn[i];
    xd1[i] = c * xdn[i];
}
// x_a = x_n + a (x_1 - x_n)
__global__ void intermediate_k(int64_t n, const double* __restrict__ xn, const double* __restrict__ x1, double a,
                               double* __restrict__ xa) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xa[i] = xn[i] + a * (x1[i] - xn[i]);
}
// R_k = u_dot(alpha_m) - v(alpha_f) on the velocity rows of solid nodes (zero elsewhere)
__global__ void kinematic_residual_k(int64_t nb, const uint8_t* __restrict__ solid, const double* __restrict__ usdn,
                                     const double* __restrict__ usd1, double am, const double* __restrict__ yaf,
                                     double* __restrict__ Rk) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t o = 3 * r + c;
        Rk[o] = solid[r] ? (usdn[o] + am * (usd1[o] - usdn[o])) - yaf[4 * r + c] : 0.0;
    }
}
// steps 1 and 2: du_dot = (alpha_f gamma dt / alpha_m) dv_dot - R_k / alpha_m;
// u_dot += du_dot; u += gamma dt du_dot   (solid rows)
__global__ void solid_update_k(int64_t nb, const uint8_t* __restrict__ solid, const double* __restrict__ dvd,
                               const double* __restrict__ Rk, double c_v, double inv_am, double gdt,
                               double* __restrict__ usd1, double* __restrict__ us1) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb || !solid[r]) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t o = 3 * r + c;
        const double du = c_v * dvd[o] - inv_am * Rk[o];
        usd1[o] += du;
        us1[o] += gdt * du;
    }
}
// the Dirichlet data of the mesh motion: the solid displacement on mesh nodes of solid rows, zero
// on the other Dirichlet nodes and on free nodes
__global__ void mesh_dirichlet_k(int64_t nL, const uint8_t* __restrict__ mmask, const int32_t* __restrict__ bop,
                                 const uint8_t* __restrict__ solid, const double* __restrict__ us,
                                 double* __restrict__ uD) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nL) return;
    const int64_t r = bop[i];
    const bool from_solid = mmask[i] && solid[r];
#pragma unroll
    for (int c = 0; c < 3; ++c) uD[3 * i + c] = from_solid ? us[3 * r + c] : 0.0;
}
// right-hand side of the eliminated mesh system: the data on Dirichlet nodes, minus the lifting
// (L_full u_D) on free nodes
__global__ void mesh_rhs_k(int64_t nL, const uint8_t* __restrict__ mmask, const double* __restrict__ uD,
                           const double* __restrict__ lift, double* __restrict__ b) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 3 * nL) return;
    b[o] = mmask[o / 3] ? uD[o] : -lift[o];
}
// step 4: v_hat = (u_hat_1 - u_hat_n) / (gamma dt) + ((gamma - 1) / gamma) v_hat_n
__global__ void mesh_velocity_k(int64_t n, const double* __restrict__ mun, const double* __restrict__ mu1,
                                const double* __restrict__ mvn, double inv_gdt, double c, double* __restrict__ mv1) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mv1[i] = (mu1[i] - mun[i]) * inv_gdt + c * mvn[i];
}
// step 7: R = K_rate (y_dot(alpha_m) - (f, 0)) + K_state y(alpha_f) + K_disp (u(alpha_f), 0), one
// thread per block row, blocks in column order
__global__ void __launch_bounds__(256) residual_k(int64_t nb, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ Kr,
                                                  const double* __restrict__ Ks, const double* __restrict__ Kd,
                                                  const double* __restrict__ ydam, const double* __restrict__ f,
                                                  const double* __restrict__ yaf, const double* __restrict__ uaf,
                                                  double* __restrict__ R) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) {
        const int64_t c = ci[q];
        double w[4], y[4], u[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[j] = ydam[4 * c + j] - ((f != nullptr && j < 3) ? f[3 * c + j] : 0.0);
            y[j] = yaf[4 * c + j];
            u[j] = j < 3 ? uaf[3 * c + j] : 0.0;
        }
        const double* kr = Kr + 16 * (int64_t)q;
        const double* ks = Ks + 16 * (int64_t)q;
        const double* kd = Kd + 16 * (int64_t)q;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) t += kr[4 * i + j] * w[j] + ks[4 * i + j] * y[j] + kd[4 * i + j] * u[j];
            acc[i] += t;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) R[4 * r + i] = acc[i];
}
__global__ void scale_k(int64_t n, const double* __restrict__ x, double a, double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}
// step 10: y_dot += d;  y += gamma dt d; the velocity-rate increment of solid rows is kept for step 1
__global__ void state_update_k(int64_t nb, const double* __restrict__ d, double gdt, const uint8_t* __restrict__ solid,
                               double* __restrict__ yd1, double* __restrict__ y1, double* __restrict__ dvd) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t o = 4 * r + j;
        yd1[o] += d[o];
        y1[o] += gdt * d[o];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) dvd[3 * r + c] = solid[r] ? d[4 * r + c] : 0.0;
}

void launch_check(const char* what) { check_launch(what); }
inline unsigned blocks(int64_t n) { return (unsigned)cdiv(n > 0 ? n : 1, 256); }

scr_status fail_step(const std::exception& e) { return status_of(e); }

// the four operator forms at dt, and (re)set up or update the hierarchies of the tangent
void assemble_all(scr_stepper* S, double dt, bool first, hipStream_t s) {
    assemble_form(S->asmb, FORM_TANGENT, dt, nullptr, S->Kt, s);
    assemble_form(S->asmb, FORM_RATE, dt, nullptr, S->Kr, s);
    assemble_form(S->asmb, FORM_STATE, dt, nullptr, S->Ks, s);
    assemble_form(S->asmb, FORM_DISP, dt, nullptr, S->Kd, s);
    scr_bsr K{(int32_t)S->nb, 4, S->nnzb, S->rp, S->ci, S->Kt};
    scr_status rc = first ? amg_setup(S->sctx, SCR_SYSTEM, &K, S->coords, &S->ao, s, &S->h)
                          : amg_update(S->h, &K, nullptr, s);
    if (rc != SCR_OK) throw Error(rc, std::string("corrector tangent: ") + scr_last_error());
    S->dt = dt;
}

}  // namespace

extern "C" {

void scr_default_corrector_opts(scr_corrector_opts* o) {
    o->max_correctors = 10;
    o->tol_R = 1e-6;
    o->tol_A = 1e-14;
    o->mesh_tol = 1e-10;
}

scr_status scr_stepper_create(scr_ctx* ctx, scr_assembler* asmb, const scr_bsr* L, const double* L_full,
                              const uint8_t* mesh_mask, const int32_t* blk_of_phys, const uint8_t* solid_rows,
                              const double* coords, double dt0, const scr_amg_opts* amg, const scr_solve_opts* solve,
                              const scr_corrector_opts* copts, void* stream, scr_stepper** out) {
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<scr_stepper> S;
    try {
        if (!ctx || !asmb || !L || !L_full || !mesh_mask || !blk_of_phys || !solid_rows || !coords || !out)
            throw Error(SCR_E_INVALID, "NULL argument");
        *out = nullptr;
        if (!(dt0 > 0.0) || !std::isfinite(dt0)) throw Error(SCR_E_INVALID, "dt must be positive");
        if (L->bs != 1 || L->n_brows < 1 || !L->row_ptr || !L->col_idx || !L->val)
            throw Error(SCR_E_INVALID, "L must be a scalar matrix");
        HIPCHK(hipSetDevice(ctx->c.device));
        S.reset(new scr_stepper());
        S->sctx = ctx;
        S->ctx = &ctx->c;
        S->ar.reset(new Arena(&ctx->c, s));
        Arena& ar = *S->ar;
        S->asmb = asmb;
        S->nb = scr_assembler_nbrows(asmb);
        S->nnzb = scr_assembler_nnzb(asmb);
        S->nL = L->n_brows;
        if (amg) S->ao = *amg; else scr_default_amg_opts(&S->ao);
        if (solve) S->so = *solve; else scr_default_solve_opts(&S->so);
        if (copts) S->co = *copts; else scr_default_corrector_opts(&S->co);
        if (S->co.max_correctors < 1 || !(S->co.tol_R > 0.0) || !(S->co.tol_A >= 0.0) || !(S->co.mesh_tol > 0.0))
            throw Error(SCR_E_INVALID, "corrector options out of range");
        const double rho = asmb_rho_inf(asmb);
        S->am = 0.5 * (3.0 - rho) / (1.0 + rho);
        S->af = 1.0 / (1.0 + rho);
        S->gam = 1.0 / (1.0 + rho);
        const int64_t nb = S->nb, nL = S->nL;
        // the tangent's pattern (the assembler's) and the inputs the steps need
        S->rp = ar.make<int32_t>(nb + 1);
        S->ci = ar.make<int32_t>(S->nnzb);
        asmb_pattern(asmb, S->rp, S->ci, s);
        S->coords = ar.make<double>(3 * nb);
        copy_dev(S->coords, coords, 3 * nb * sizeof(double), s);
        S->solid_rows = ar.make<uint8_t>(nb);
        copy_dev(S->solid_rows, solid_rows, nb, s);
        S->mesh_mask = ar.make<uint8_t>(nL);
        copy_dev(S->mesh_mask, mesh_mask, nL, s);
        S->blk_of_phys = ar.make<int32_t>(nL);
        copy_dev(S->blk_of_phys, blk_of_phys, nL * sizeof(int32_t), s);
        std::vector<int32_t> hb(nL);
        HIPCHK(hipMemcpyAsync(hb.data(), blk_of_phys, nL * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int32_t b : hb)
            if (b < 0 || b >= nb) throw Error(SCR_E_INVALID, "blk_of_phys out of range");
        for (double** p : {&S->Kt, &S->Kr, &S->Ks, &S->Kd}) *p = ar.make<double>(16 * S->nnzb);
        assemble_all(S.get(), dt0, true, s);
        scr_status rc = amg_setup(ctx, MESH_SYSTEM, L, nullptr, &S->ao, s, &S->hm);
        if (rc != SCR_OK) throw Error(rc, std::string("mesh hierarchy: ") + scr_last_error());
        DBsr Lf;
        Lf.nr = Lf.nc = nL; Lf.br = Lf.bc = 1; Lf.nnzb = L->nnzb;
        Lf.rp = const_cast<int32_t*>(L->row_ptr); Lf.ci = const_cast<int32_t*>(L->col_idx);
        Lf.v = const_cast<double*>(L_full);
        S->Lfull = sell_from_bsr<double>(Lf, ar, s);
        for (double** p : {&S->yn, &S->y1, &S->ydn, &S->yd1, &S->yaf, &S->ydam, &S->R, &S->rhs, &S->dyd})
            *p = ar.make<double>(4 * nb);
        for (double** p : {&S->usn, &S->us1, &S->usdn, &S->usd1, &S->uaf, &S->Rk, &S->dvd}) *p = ar.make<double>(3 * nb);
        for (double** p : {&S->mun, &S->mu1, &S->mvn, &S->mv1, &S->uD, &S->lift, &S->bm}) *p = ar.make<double>(3 * nL);
        // at rest
        zero_dev(S->yn, 4 * nb * sizeof(double), s);
        zero_dev(S->ydn, 4 * nb * sizeof(double), s);
        zero_dev(S->usn, 3 * nb * sizeof(double), s);
        zero_dev(S->usdn, 3 * nb * sizeof(double), s);
        zero_dev(S->mun, 3 * nL * sizeof(double), s);
        zero_dev(S->mvn, 3 * nL * sizeof(double), s);
        S->red.init(4 * nb, ar, s);
        S->slot.h = ctx->c.pinned.get();
        S->slot.d = PinnedPool::device_ptr(S->slot.h);
        S->slot.h[15] = 0.0;
        HIPCHK(hipStreamSynchronize(s));
        *out = S.release();
        return SCR_OK;
    } catch (const std::exception& e) {
        if (S) {
            (void)hipStreamSynchronize(s);
            if (S->h) scr_handle_destroy(S->h);
            if (S->hm) scr_handle_destroy(S->hm);
            if (S->slot.h) S->ctx->pinned.put(S->slot.h);
            S->ar.reset();
        }
        return fail_step(e);
    }
}

scr_status scr_stepper_state(scr_stepper* S, int which, double* dst, int set, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!S || !dst) throw Error(SCR_E_INVALID, "NULL argument");
        HIPCHK(hipSetDevice(S->ctx->device));
        double* src = nullptr;
        int64_t n = 0;
        switch (which) {
            case SCR_STATE_Y: src = S->yn; n = 4 * S->nb; break;
            case SCR_STATE_YDOT: src = S->ydn; n = 4 * S->nb; break;
            case SCR_STATE_U_SOLID: src = S->usn; n = 3 * S->nb; break;
            case SCR_STATE_UDOT_SOLID: src = S->usdn; n = 3 * S->nb; break;
            case SCR_STATE_U_MESH: src = S->mun; n = 3 * S->nL; break;
            case SCR_STATE_V_MESH: src = S->mvn; n = 3 * S->nL; break;
            default: throw Error(SCR_E_INVALID, "unknown state field");
        }
        if (set) copy_dev(src, dst, n * sizeof(double), s);
        else copy_dev(dst, src, n * sizeof(double), s);
        HIPCHK(hipStreamSynchronize(s));
        return SCR_OK;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        return fail_step(e);
    }
}

scr_status scr_step(scr_stepper* S, double dt, const double* f, void* stream, scr_step_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    scr_step_stats st{};
    try {
        if (!S) throw Error(SCR_E_INVALID, "NULL stepper");
        if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(SCR_E_INVALID, "dt must be positive");
        HIPCHK(hipSetDevice(S->ctx->device));
        const int64_t nb = S->nb, nL = S->nL;
        if (dt != S->dt) {
            assemble_all(S, dt, false, s);
            st.resetups = 1;
        }
        const double am = S->am, af = S->af, gam = S->gam;
        const double cpred = (gam - 1.0) / gam, gdt = gam * dt, afgdt = af * gam * dt;
        // predictor
        predictor_k<<<blocks(4 * nb), 256, 0, s>>>(4 * nb, S->yn, S->ydn, S->y1, S->yd1, cpred);
        predictor_k<<<blocks(3 * nb), 256, 0, s>>>(3 * nb, S->usn, S->usdn, S->us1, S->usd1, cpred);
        predictor_k<<<blocks(3 * nL), 256, 0, s>>>(3 * nL, S->mun, S->mvn, S->mu1, S->mv1, cpred);
        zero_dev(S->dvd, 3 * nb * sizeof(double), s);
        launch_check("predictor");
        scr_solve_opts mo = S->so;
        mo.tol = S->co.mesh_tol;
        mo.max_it = std::max(S->so.max_it, 500);
        double res0 = 0.0;
        for (int l = 1; l <= S->co.max_correctors; ++l) {
            st.correctors = l;
            // steps 1 and 2: du_dot_s from the previous corrector's velocity-rate increment and the
            // kinematic residual at the iterate before that increment (at l = 1: the predictor and a
            // zero increment); afterwards R_k is recomputed (zero up to rounding) for the next corrector
            if (l == 1) {
                intermediate_k<<<blocks(4 * nb), 256, 0, s>>>(4 * nb, S->yn, S->y1, af, S->yaf);
                kinematic_residual_k<<<blocks(nb), 256, 0, s>>>(nb, S->solid_rows, S->usdn, S->usd1, am, S->yaf, S->Rk);
            }
            solid_update_k<<<blocks(nb), 256, 0, s>>>(nb, S->solid_rows, S->dvd, S->Rk, afgdt / am, 1.0 / am, gdt,
                                                      S->usd1, S->us1);
            intermediate_k<<<blocks(4 * nb), 256, 0, s>>>(4 * nb, S->yn, S->y1, af, S->yaf);
            kinematic_residual_k<<<blocks(nb), 256, 0, s>>>(nb, S->solid_rows, S->usdn, S->usd1, am, S->yaf, S->Rk);
            // steps 3 and 4: mesh motion with the solid displacement as Dirichlet data, mesh velocity
            mesh_dirichlet_k<<<blocks(nL), 256, 0, s>>>(nL, S->mesh_mask, S->blk_of_phys, S->solid_rows, S->us1, S->uD);
            sell_mv3<double>(S->Lfull, S->uD, nullptr, S->lift, 0, s);
            mesh_rhs_k<<<blocks(3 * nL), 256, 0, s>>>(nL, S->mesh_mask, S->uD, S->lift, S->bm);
            launch_check("mesh data");
            scr_stats ms{};
            scr_status rm = mesh_motion_solve(S->hm, S->bm, S->mu1, &mo, s, &ms);
            if (rm < 0) throw Error(rm, std::string("mesh motion: ") + scr_last_error());
            st.mesh_its += ms.outer_it;
            mesh_velocity_k<<<blocks(3 * nL), 256, 0, s>>>(3 * nL, S->mun, S->mu1, S->mvn, 1.0 / gdt, cpred, S->mv1);
            // step 7: residual of the balance equations at the intermediate states (y(alpha_f) is current)
            intermediate_k<<<blocks(4 * nb), 256, 0, s>>>(4 * nb, S->ydn, S->yd1, am, S->ydam);
            intermediate_k<<<blocks(3 * nb), 256, 0, s>>>(3 * nb, S->usn, S->us1, af, S->uaf);
            residual_k<<<blocks(nb), 256, 0, s>>>(nb, S->rp, S->ci, S->Kr, S->Ks, S->Kd, S->ydam, f, S->yaf, S->uaf, S->R);
            launch_check("residual");
            // step 8: stopping test
            const double res = device_norm(S->R, 4 * nb, S->red, S->slot, s);
            if (!std::isfinite(res)) throw Error(SCR_E_BREAKDOWN, "non-finite corrector residual");
            if (l == 1) res0 = res;
            st.res0 = res0;
            st.res = res;
            if ((res0 > 0.0 && res / res0 <= S->co.tol_R) || res <= S->co.tol_A) {
                st.converged = 1;
                break;
            }
            if (l == S->co.max_correctors) break;
            // step 9: the corrector system (the tangent divided by alpha_f gamma dt)
            scale_k<<<blocks(4 * nb), 256, 0, s>>>(4 * nb, S->R, -1.0 / afgdt, S->rhs);
            launch_check("corrector rhs");
            scr_stats ls{};
            scr_status rl = scr_solve(S->h, S->rhs, S->dyd, &S->so, s, &ls);
            if (rl < 0) throw Error(rl, std::string("corrector solve: ") + scr_last_error());
            st.linear_its += ls.outer_it;
            // steps 10 and 11 (the intermediate states are formed at the top of the next corrector)
            state_update_k<<<blocks(nb), 256, 0, s>>>(nb, S->dyd, gdt, S->solid_rows, S->yd1, S->y1, S->dvd);
            launch_check("state update");
        }
        // the iterate becomes the state at t_{n+1}
        std::swap(S->yn, S->y1); std::swap(S->ydn, S->yd1);
        std::swap(S->usn, S->us1); std::swap(S->usdn, S->usd1);
        std::swap(S->mun, S->mu1); std::swap(S->mvn, S->mv1);
        HIPCHK(hipStreamSynchronize(s));
        st.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = st;
        return st.converged ? SCR_OK : SCR_NOT_CONVERGED;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        if (stats) *stats = st;
        return fail_step(e);
    }
}

scr_status scr_stepper_destroy(scr_stepper* S) {
    if (!S) return SCR_OK;
    hipStream_t s = S->ar ? S->ar->stream() : nullptr;
    (void)hipStreamSynchronize(s);
    if (S->h) scr_handle_destroy(S->h);
    if (S->hm) scr_handle_destroy(S->hm);
    if (S->slot.h) S->ctx->pinned.put(S->slot.h);
    S->red.release(*S->ar);
    delete S;
    return SCR_OK;
}

}  // extern "C"
