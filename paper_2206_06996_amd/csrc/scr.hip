// scr.hip -- handles, the SCR preconditioner (Appendix B, Algorithms 1 and 2), the outer FGMRES
// (Sec. 5.2.1), the mesh-motion CG (Sec. 5.2.2) and the extern "C" boundary declared in scr.h.
#include <chrono>
#include <cmath>
#include <memory>

#include "solver.h"

using namespace scr;

namespace scr {
static thread_local std::string g_last_error;
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace scr

// Device scratch of mesh_motion_solve_noalloc (the three-column CG's workspace), one copy per GPU,
// held until the process ends.  Host code uses only the per-device address from
// hipGetSymbolAddress (noalloc_scratch), never this name.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = int64_t(32) << 20;     // 256 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// the address of this device's copy of `scratch`; the device must be current.  Taken once per
// device (at context creation).
double* noalloc_scratch(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) throw Error(SCR_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw Error(SCR_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    return g_scratch_ptr[device];
}
}  // namespace

struct scr_handle {
    Ctx* ctx = nullptr;
    int kind = SCR_SYSTEM;
    scr_amg_opts opts{};
    std::unique_ptr<Arena> ar;
    int64_t nb = 0;
    // SCR system (FP64 setup form; A, G, D, C share K's index arrays)
    DBsr K, A, G, D, C, Sh;
    DSell<double> Ks, As, Gs, Ds, Cs, Ls, Shs;   // Shs: S^ for SIMPLE, built on first use
    double* B = nullptr;
    double* dvec = nullptr;                       // the diagonal d used in S^ (3n)
    std::unique_ptr<Hierarchy> hA, hS, hL;
    std::unique_ptr<Gmres> gOuter, gA, gS;
    // SCR_MIXED_FP32_INNER: Algorithm 2's inner A solve on FP32 vectors (FP32 A of the hierarchy)
    std::unique_ptr<GmresT<float>> gA32;
    float *xbar32 = nullptr, *xtil32 = nullptr;
    int restart = 0, restart_inner = 0;
    double *bs = nullptr, *xs = nullptr, *yhat = nullptr, *tv = nullptr, *tp = nullptr, *xbar = nullptr,
           *xtil = nullptr;
    // mesh motion: the three-column CG's workspace (allocated on the first solve) and its status slot
    double* mws = nullptr;
    StatusSlot mslot;
    scr_stats st{};
    scr_solve_opts so{};
    bool broken = false;                          // a failed amg_update left the hierarchies half-updated
    // outlet coupling (scr_set_outlets): outlet k adds m_k a_k a_k^T to the velocity block; entry e
    // of the concatenated list names block row out_blk[e], outlet out_id[e] and a_k there (3)
    int n_out = 0;
    int64_t n_oe = 0;
    int32_t *out_blk = nullptr, *out_id = nullptr;
    int64_t* out_off = nullptr;
    double *out_a = nullptr, *out_m = nullptr, *out_s = nullptr;
};

namespace {

// s_k = m_k * (a_k . x_v): one workgroup per outlet, its entries strided over the threads and the
// partial sums added by a fixed LDS tree
template <typename T>
__global__ void __launch_bounds__(256) outlet_dot_k(const int64_t* __restrict__ off, const int32_t* __restrict__ blk,
                                                    const double* __restrict__ a, const double* __restrict__ m,
                                                    const T* __restrict__ x, double* __restrict__ sk) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int64_t e = off[k] + threadIdx.x; e < off[k + 1]; e += 256) {
        const int64_t b = blk[e];
        acc += a[3 * e] * (double)x[3 * b] + a[3 * e + 1] * (double)x[3 * b + 1] + a[3 * e + 2] * (double)x[3 * b + 2];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sk[k] = m[k] * red[0];
}
// y_v += s_k a_k (block rows are distinct across all outlets, so entries never collide)
template <typename T>
__global__ void outlet_axpy_k(int64_t ne, const int32_t* __restrict__ blk, const int32_t* __restrict__ id,
                              const double* __restrict__ a, const double* __restrict__ sk, T* __restrict__ y) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const double c = sk[id[e]];
    const int64_t b = blk[e];
    for (int i = 0; i < 3; ++i) y[3 * b + i] = (T)((double)y[3 * b + i] + c * a[3 * e + i]);
}

// y_v += sum_k m_k a_k (a_k . x_v) on velocity vectors (node-interleaved, 3 per block row)
template <typename T>
void apply_outlets(const scr_handle* h, const T* xv, T* yv, hipStream_t s) {
    if (h->n_out == 0) return;
    outlet_dot_k<T><<<h->n_out, 256, 0, s>>>(h->out_off, h->out_blk, h->out_a, h->out_m, xv, h->out_s);
    outlet_axpy_k<T><<<cdiv(h->n_oe, 256), 256, 0, s>>>(h->n_oe, h->out_blk, h->out_id, h->out_a, h->out_s, yv);
    check_launch("outlets");
}

struct MatOp : Op {
    const DSell<double>* M;
    explicit MatOp(const DSell<double>* m) : M(m) {}
    void apply(const double* x, double* y, hipStream_t s) override { sell_mv<double>(*M, x, nullptr, y, 0, s); }
};
// the scalar mesh Laplacian and AMG(L) on three node-interleaved columns
struct MatOp3 : Op {
    const DSell<double>* M;
    explicit MatOp3(const DSell<double>* m) : M(m) {}
    void apply(const double* x, double* y, hipStream_t s) override { sell_mv3<double>(*M, x, nullptr, y, 0, s); }
};
struct VOp3 : Op {
    Hierarchy* H;
    explicit VOp3(Hierarchy* h) : H(h) {}
    void apply(const double* x, double* y, hipStream_t s) override { H->vcycle3(x, y, s); }
};
// K with the outlet coupling, on split vectors (the velocity part leads)
struct KOp : Op {
    const scr_handle* h;
    explicit KOp(const scr_handle* hh) : h(hh) {}
    void apply(const double* x, double* y, hipStream_t s) override {
        sell_mv_split4(h->Ks, x, nullptr, y, 0, s);
        apply_outlets(h, x, y, s);
    }
};
// the velocity block A with the outlet coupling
struct AOp : Op {
    const scr_handle* h;
    explicit AOp(const scr_handle* hh) : h(hh) {}
    void apply(const double* x, double* y, hipStream_t s) override {
        sell_mv<double>(h->As, x, nullptr, y, 0, s);
        apply_outlets(h, x, y, s);
    }
};
// the same on FP32 vectors, with the FP32 copy of A that level 0 of the mixed hierarchy holds
struct AOp32 : OpT<float> {
    const scr_handle* h;
    explicit AOp32(const scr_handle* hh) : h(hh) {}
    void apply(const float* x, float* y, hipStream_t s) override {
        sell_mv<float>(*h->hA->level0_f(), x, nullptr, y, 0, s);
        apply_outlets(h, x, y, s);
    }
};
struct VOp32 : OpT<float> {
    Hierarchy* H;
    int64_t* count;
    VOp32(Hierarchy* hh, int64_t* c) : H(hh), count(c) {}
    void apply(const float* x, float* y, hipStream_t s) override {
        H->vcycle_f(x, y, s);
        ++*count;
    }
};
struct VOp : Op {
    Hierarchy* H;
    int64_t* count;
    VOp(Hierarchy* h, int64_t* c) : H(h), count(c) {}
    void apply(const double* x, double* y, hipStream_t s) override {
        H->vcycle(x, y, s);
        ++*count;
    }
};

// Algorithm 2: y = S x_p = C x_p - D A^-1 (G x_p), A^-1 by GMRES + AMG(A) to delta_I
struct SchurOp : Op {
    scr_handle* h;
    explicit SchurOp(scr_handle* hh) : h(hh) {}
    void apply(const double* xp, double* y, hipStream_t s) override {
        sell_mv<double>(h->Gs, xp, nullptr, h->xbar, 0, s);
        KStat k;
        if (h->gA32) {
            // SCR_MIXED_FP32_INNER: the inner solve to delta_I on FP32 vectors, FP32 A and V-cycle
            const int64_t n3 = 3 * h->nb;
            cast_d2f(h->xbar, h->xbar32, n3, s);
            AOp32 aop(h);
            VOp32 pa(h->hA.get(), &h->st.vcycles_A);
            k = h->gA32->solve(aop, pa, h->xbar32, h->xtil32, h->so.tol_I, h->so.max_it_I, false, false, s);
            cast_f2d(h->xtil32, h->xtil, n3, s);
        } else {
            AOp aop(h);
            VOp pa(h->hA.get(), &h->st.vcycles_A);
            k = h->gA->solve(aop, pa, h->xbar, h->xtil, h->so.tol_I, h->so.max_it_I, false, false, s);
        }
        h->st.calls_I++;
        h->st.its_I += k.iters;
        sell_mv<double>(h->Cs, xp, nullptr, y, 0, s);
        sell_mv<double>(h->Ds, h->xtil, nullptr, y, 3, s);
    }
};

// Algorithm 1 (step 2 read as r_p <- r_p - D y^_v):  y = P_SCR^-1 r on split vectors
struct ScrPrec : Op {
    scr_handle* h;
    explicit ScrPrec(scr_handle* hh) : h(hh) {}
    void apply(const double* r, double* y, hipStream_t s) override {
        const int64_t n = h->nb;
        const double* rv = r;
        const double* rp = r + 3 * n;
        double* yv = y;
        double* yp = y + 3 * n;
        AOp aop(h);
        VOp pa(h->hA.get(), &h->st.vcycles_A);
        KStat k = h->gA->solve(aop, pa, rv, h->yhat, h->so.tol_A, h->so.max_it_A, false, false, s);
        h->st.calls_A++;
        h->st.its_A += k.iters;
        sell_mv<double>(h->Ds, h->yhat, rp, h->tp, 1, s);            // r_p - D y^_v
        SchurOp sop(h);
        VOp ps(h->hS.get(), &h->st.vcycles_S);
        k = h->gS->solve(sop, ps, h->tp, yp, h->so.tol_S, h->so.max_it_S, false, false, s);
        h->st.calls_S++;
        h->st.its_S += k.iters;
        sell_mv<double>(h->Gs, yp, rv, h->tv, 1, s);                 // r_v - G y_p
        k = h->gA->solve(aop, pa, h->tv, yv, h->so.tol_A, h->so.max_it_A, false, false, s);
        h->st.calls_A++;
        h->st.its_A += k.iters;
    }
};

// y_v = y*_v - (G y_p) / d   (the SIMPLE velocity update; division as in the definition)
__global__ void simple_update_k(int64_t n, const double* __restrict__ ystar, const double* __restrict__ t,
                                const double* __restrict__ d, double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = ystar[i] - t[i] / d[i];
}

// SIMPLE / SIMPLEC (Sec. 5.2.1): P = [I 0; D A^-1 I] [A 0; 0 S^] [I d^-1 G; 0 I];
//   y*_v = A^-1 r_v (GMRES + AMG(A), delta_A);  y_p = S^^-1 (r_p - D y*_v) (GMRES + AMG(S^) on the
//   explicit S^, delta_S: no inner-level solver);  y_v = y*_v - d^-1 (G y_p)
struct SimplePrec : Op {
    scr_handle* h;
    explicit SimplePrec(scr_handle* hh) : h(hh) {}
    void apply(const double* r, double* y, hipStream_t s) override {
        const int64_t n = h->nb;
        const double* rv = r;
        const double* rp = r + 3 * n;
        double* yv = y;
        double* yp = y + 3 * n;
        AOp aop(h);
        VOp pa(h->hA.get(), &h->st.vcycles_A);
        KStat k = h->gA->solve(aop, pa, rv, h->yhat, h->so.tol_A, h->so.max_it_A, false, false, s);
        h->st.calls_A++;
        h->st.its_A += k.iters;
        sell_mv<double>(h->Ds, h->yhat, rp, h->tp, 1, s);            // r_p - D y*_v
        MatOp shop(&h->Shs);
        VOp ps(h->hS.get(), &h->st.vcycles_S);
        k = h->gS->solve(shop, ps, h->tp, yp, h->so.tol_S, h->so.max_it_S, false, false, s);
        h->st.calls_S++;
        h->st.its_S += k.iters;
        sell_mv<double>(h->Gs, yp, nullptr, h->tv, 0, s);            // G y_p
        simple_update_k<<<cdiv(3 * n, 256), 256, 0, s>>>(3 * n, h->yhat, h->tv, h->dvec, yv);
        check_launch("simple_update");
    }
};

void ensure_simple(scr_handle* h, hipStream_t s) {
    if (h->Shs.nslices == 0 && h->Sh.nr > 0) h->Shs = sell_from_bsr<double>(h->Sh, *h->ar, s);
}

scr_status fail(const std::exception& e) { return status_of(e); }

void ensure_workspaces(scr_handle* h, const scr_solve_opts& o, hipStream_t s) {
    if (o.restart < 1 || o.restart > 63 || o.restart_inner < 1 || o.restart_inner > 63)
        throw Error(SCR_E_INVALID, "restart lengths must be in [1, 63]");
    h->ar->set_stream(s);
    if (h->kind == SCR_SYSTEM) {
        if (!h->gOuter || h->restart != o.restart) {
            h->gOuter.reset();
            h->gOuter.reset(new Gmres(4 * h->nb, o.restart, *h->ar, s));
            h->restart = o.restart;
        }
        if (!h->gA || h->restart_inner != o.restart_inner) {
            h->gA.reset(new Gmres(3 * h->nb, o.restart_inner, *h->ar, s));
            h->gS.reset(new Gmres(h->nb, o.restart_inner, *h->ar, s));
            h->gA32.reset();
            if (h->opts.precision == SCR_MIXED_FP32_INNER && h->hA->level0_f())
                h->gA32.reset(new GmresT<float>(3 * h->nb, o.restart_inner, *h->ar, s));
            h->restart_inner = o.restart_inner;
        }
        if (h->gA32 && !h->xbar32) {
            h->xbar32 = h->ar->make<float>(3 * h->nb);
            h->xtil32 = h->ar->make<float>(3 * h->nb);
        }
    } else if (!h->mws) {
        h->mws = h->ar->make<double>(Pcg3::workspace_doubles(h->nb));
    }
}

// The mesh-motion solve of Sec. 5.2.2 on the three interleaved columns: CG (flexible CG for an FP32
// hierarchy or on request) with one product with L and one V-cycle of AMG(L) per iteration for all
// three columns; ws holds Pcg3::workspace_doubles(n) doubles.  Fills the handle's stats.
bool mesh_solve_run(scr_handle* h, const double* b, double* x, const scr_solve_opts& o, double* ws, hipStream_t s) {
    MatOp3 lop(&h->Ls);
    VOp3 pl(h->hL.get());
    const bool flexible = o.flexible_cg || h->opts.precision != SCR_FP64;
    const int64_t v0 = h->hL->vcycles;
    Pcg3 cg(h->nb, ws, &h->mslot);
    Pcg3::Result k = cg.solve(lop, pl, b, x, o.tol, o.max_it, flexible, s);
    bool ok = true;
    for (int c = 0; c < 3; ++c) {
        h->st.mesh_its[c] = k.iters[c];
        h->st.mesh_rel[c] = k.rel[c];
        ok &= k.converged[c];
        if (k.iters[c] > h->st.outer_it) h->st.outer_it = (int)k.iters[c];
        if (k.rel[c] > h->st.rel_res_true) h->st.rel_res_true = k.rel[c];
    }
    h->st.vcycles_L = h->hL->vcycles - v0;
    return ok;
}

// flag = 1 if the pattern (rp, ci) differs from the stored one (rp already known to be in range)
__global__ void pattern_diff_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const int32_t* __restrict__ rp0, const int32_t* __restrict__ ci0, int* __restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nr) return;
    if (rp[i] != rp0[i]) { atomicOr(flag, 1); return; }
    if (i == nr) return;
    for (int32_t q = rp0[i]; q < rp0[i + 1]; ++q)
        if (ci[q] != ci0[q]) { atomicOr(flag, 1); return; }
}

void check_opts(const scr_solve_opts& o) {
    if (!(o.tol > 0) || !(o.tol_A > 0) || !(o.tol_S > 0) || !(o.tol_I > 0) || o.max_it < 1 || o.max_it_A < 1 ||
        o.max_it_S < 1 || o.max_it_I < 1)
        throw Error(SCR_E_INVALID, "tolerances must be positive and iteration limits >= 1");
    if (o.precond != SCR_PRECOND_SCR && o.precond != SCR_PRECOND_SIMPLE)
        throw Error(SCR_E_INVALID, "precond must be SCR_PRECOND_SCR or SCR_PRECOND_SIMPLE");
}

}  // namespace

// Chebyshev degree of AMG(S^) when the options leave it to the size of S^ (measured on the test
// tubes and the Y: each Schur iteration saved also saves an inner A solve of Algorithm 2, which
// pays for a stronger Schur smoother on the larger meshes, where the Schur counts grow)
static int schur_degree_by_size(int64_t n) { return n <= 1000000 ? 8 : (n <= 3000000 ? 12 : 16); }

extern "C" {

void scr_default_amg_opts(scr_amg_opts* o) {
    o->precision = SCR_FP64;
    o->theta = 0.08;
    o->smoother = SCR_SMOOTH_CHEBYSHEV;
    o->cheb_degree = 4;
    o->schur_cheb_degree = -1;
    o->schur_cheb_ratio = 100.0;
    o->cheb_ratio = 30.0;
    o->jacobi_sweeps = 2;
    o->coarse_max = 1024;
    o->max_levels = 10;
    o->max_coarse_ratio = 0.8;
    o->seed = 0;
    o->schur_diag = SCR_DIAG_A;
    o->amg_type = SCR_AMG_SA;
    o->cl_theta = 0.5;
    o->trunc = 0.3;
    o->pmax = 5;
    o->agg_levels = 2;
    o->l1_gs = 1;
}

void scr_default_solve_opts(scr_solve_opts* o) {
    o->tol = 1e-8;
    o->tol_A = o->tol_S = o->tol_I = 1e-3;
    o->max_it = o->max_it_A = o->max_it_S = o->max_it_I = 200;
    o->restart = 50;
    o->restart_inner = 30;
    o->use_x0 = 0;
    o->flexible_cg = 0;
    o->precond = SCR_PRECOND_SCR;
}

const char* scr_status_str(scr_status s) {
    switch (s) {
        case SCR_OK: return "ok";
        case SCR_NOT_CONVERGED: return "not converged";
        case SCR_E_INVALID: return "invalid input";
        case SCR_E_OOM: return "out of device memory";
        case SCR_E_HIP: return "HIP error";
        case SCR_E_BREAKDOWN: return "Krylov breakdown (non-finite value)";
        case SCR_E_UNIMPLEMENTED: return "unimplemented";
        case SCR_E_NO_DEVICE: return "no device";
    }
    return "unknown status";
}

const char* scr_last_error(void) { return g_last_error.c_str(); }

scr_status scr_ctx_create(int device, int64_t hbm_budget, scr_ctx** out) {
    try {
        if (!out) throw Error(SCR_E_INVALID, "out is NULL");
        *out = nullptr;
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) throw Error(SCR_E_NO_DEVICE, "no HIP device");
        if (device < 0 || device >= n) throw Error(SCR_E_INVALID, "device index out of range");
        HIPCHK(hipSetDevice(device));
        hipDeviceProp_t p;
        HIPCHK(hipGetDeviceProperties(&p, device));
        // keep freed stream-ordered memory in the pool (solves allocate nothing once warm)
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        (void)noalloc_scratch(device);     // this device's scratch address, once (device is current)
        auto* c = new scr_ctx();
        c->c.device = device;
        c->c.budget = hbm_budget;
        c->c.cu_count = p.multiProcessorCount;
        *out = c;
        return SCR_OK;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

void scr_ctx_destroy(scr_ctx* ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    ctx->c.cache.flush();
    ctx->c.prof.harvest();
    for (auto& p : ctx->c.prof.pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : ctx->c.prof.pool) (void)hipEventDestroy(e);
    delete ctx;
}

scr_status scr_ctx_profile(scr_ctx* ctx, int kernel) {
    if (!ctx) { set_last_error("NULL context"); return SCR_E_INVALID; }
    if (kernel != SCR_PROF_OFF && kernel != SCR_PROF_SMOOTH_A0) { set_last_error("unknown kernel"); return SCR_E_INVALID; }
    ctx->c.prof.kernel.store(kernel);
    return SCR_OK;
}

scr_status scr_ctx_profile_read(scr_ctx* ctx, int64_t* launches, double* total_ms, double* bytes) {
    if (!ctx || !launches || !total_ms || !bytes) { set_last_error("NULL argument"); return SCR_E_INVALID; }
    Profiler& p = ctx->c.prof;
    p.harvest();
    std::lock_guard<std::mutex> g(p.mu);
    *launches = p.launches; *total_ms = p.ms; *bytes = p.bytes;
    p.launches = 0; p.ms = 0.0; p.bytes = 0.0;
    return SCR_OK;
}
int64_t scr_ctx_bytes_in_use(const scr_ctx* ctx) { return ctx ? ctx->c.in_use.load() : 0; }

scr_status amg_setup(scr_ctx* ctx, int kind, const scr_bsr* K, const double* coords, const scr_amg_opts* opts,
                     void* stream, scr_handle** out) {
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<scr_handle> h;
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!ctx || !K || !out) throw Error(SCR_E_INVALID, "NULL argument");
        *out = nullptr;
        if (kind != SCR_SYSTEM && kind != MESH_SYSTEM) throw Error(SCR_E_INVALID, "unknown kind");
        int want = kind == SCR_SYSTEM ? 4 : 1;
        if (K->bs != want) throw Error(SCR_E_INVALID, "block size must be 4 (SCR_SYSTEM) or 1 (MESH_SYSTEM)");
        if (K->n_brows <= 0 || K->nnzb < K->n_brows) throw Error(SCR_E_INVALID, "empty matrix or missing diagonal");
        if (!K->row_ptr || !K->col_idx || !K->val) throw Error(SCR_E_INVALID, "NULL matrix array");
        if (kind == SCR_SYSTEM && !coords) throw Error(SCR_E_INVALID, "coords are required for SCR_SYSTEM");
        HIPCHK(hipSetDevice(ctx->c.device));
        h.reset(new scr_handle());
        h->ctx = &ctx->c;
        h->kind = kind;
        if (opts) h->opts = *opts;
        else scr_default_amg_opts(&h->opts);
        const scr_amg_opts& o = h->opts;
        if (o.precision != SCR_FP64 && o.precision != SCR_MIXED && o.precision != SCR_MIXED_FP32_INNER)
            throw Error(SCR_E_INVALID, "precision");
        if (!(o.theta > 0) || o.coarse_max < 1 || o.max_levels < 1 || o.cheb_degree < 1 || o.jacobi_sweeps < 1 ||
            !(o.cheb_ratio > 1) || !(o.max_coarse_ratio > 0) || o.schur_cheb_degree < -1 ||
            !(o.schur_cheb_ratio == 0.0 || o.schur_cheb_ratio > 1))
            throw Error(SCR_E_INVALID, "AMG options out of range");
        if (o.amg_type != SCR_AMG_SA && o.amg_type != SCR_AMG_CLASSICAL) throw Error(SCR_E_INVALID, "amg_type");
        if (o.amg_type == SCR_AMG_CLASSICAL &&
            (!(o.cl_theta > 0 && o.cl_theta <= 1) || !(o.trunc >= 0 && o.trunc < 1) ||
             o.pmax < 1 || o.pmax > 16 || o.agg_levels < 0 || o.agg_levels > 16 ||
             (o.l1_gs != 0 && o.l1_gs != 1)))
            throw Error(SCR_E_INVALID,
                        "classical AMG: 0 < cl_theta <= 1, 0 <= trunc < 1, 1 <= pmax <= 16, 0 <= agg_levels <= 16, l1_gs 0 or 1");
        h->ar.reset(new Arena(&ctx->c, s));
        Arena& ar = *h->ar;
        const int64_t nb = K->n_brows;
        h->nb = nb;
        // row_ptr endpoints first, so that the validation kernel never reads outside col_idx
        int32_t ends[2];
        HIPCHK(hipMemcpyAsync(&ends[0], K->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&ends[1], K->row_ptr + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (ends[0] != 0 || ends[1] != K->nnzb) throw Error(SCR_E_INVALID, "row_ptr[0] != 0 or row_ptr[n] != nnzb");
        int bits = validate_bsr(nb, K->bs, K->nnzb, K->row_ptr, K->col_idx, K->val, ar, s);
        if (bits) {
            std::string m = "malformed matrix:";
            if (bits & 1) m += " row_ptr";
            if (bits & 2) m += " column-out-of-range";
            if (bits & 4) m += " unsorted-or-duplicate-columns";
            if (bits & 8) m += " missing-diagonal";
            if (bits & 16) m += " non-finite-value";
            if (bits & 32) m += " zero-diagonal";
            throw Error(SCR_E_INVALID, m);
        }
        DBsr& Km = h->K;
        Km.nr = Km.nc = nb; Km.br = Km.bc = K->bs; Km.nnzb = K->nnzb;
        Km.rp = ar.make<int32_t>(nb + 1);
        Km.ci = ar.make<int32_t>(K->nnzb);
        Km.v = ar.make<double>(K->nnzb * K->bs * K->bs);
        copy_dev(Km.rp, K->row_ptr, (nb + 1) * sizeof(int32_t), s);
        copy_dev(Km.ci, K->col_idx, K->nnzb * sizeof(int32_t), s);
        copy_dev(Km.v, K->val, K->nnzb * K->bs * K->bs * sizeof(double), s);
        if (kind == SCR_SYSTEM) {
            split_blocks(Km, h->A, h->G, h->D, h->C, ar, s);
            if (o.schur_diag != SCR_DIAG_A && o.schur_diag != SCR_DIAG_ABSROWSUM)
                throw Error(SCR_E_INVALID, "schur_diag must be SCR_DIAG_A or SCR_DIAG_ABSROWSUM");
            h->dvec = ar.make<double>(3 * nb);
            h->Sh = schur_approx(h->A, h->G, h->D, h->C, o.schur_diag, h->dvec, ar, s);
            double* xyz = ar.make<double>(nb * 3);
            copy_dev(xyz, coords, nb * 3 * sizeof(double), s);
            h->B = ar.make<double>(nb * 18);
            rigid_modes(nb, xyz, h->B, ar, s);
            ar.free(xyz);
            Profiler* pa = ctx->c.prof.kernel.load() == SCR_PROF_SMOOTH_A0 ? &ctx->c.prof : nullptr;
            h->hA = build_hierarchy(h->A, h->B, 6, o, ar, s, pa);
            double* ones = ar.make<double>(nb);
            fill<double>(ones, 1.0, nb, s);
            // AMG(S^) with its own Chebyshev settings: its V-cycles are cheap (scalar, small), and
            // each Schur iteration saved also saves an inner A solve of Algorithm 2
            scr_amg_opts oS = o;
            const int sdeg = o.schur_cheb_degree >= 0 ? o.schur_cheb_degree : schur_degree_by_size(nb);
            if (sdeg > 0) oS.cheb_degree = sdeg;
            if (o.schur_cheb_ratio > 0) oS.cheb_ratio = o.schur_cheb_ratio;
            h->hS = build_hierarchy(h->Sh, ones, 1, oS, ar, s);
            ar.free(ones);
            h->Ks = sell_from_bsr<double>(Km, ar, s);
            h->As = sell_from_bsr<double>(h->A, ar, s);
            h->Gs = sell_from_bsr<double>(h->G, ar, s);
            h->Ds = sell_from_bsr<double>(h->D, ar, s);
            h->Cs = sell_from_bsr<double>(h->C, ar, s);
            h->bs = ar.make<double>(4 * nb);
            h->xs = ar.make<double>(4 * nb);
            h->yhat = ar.make<double>(3 * nb);
            h->tv = ar.make<double>(3 * nb);
            h->tp = ar.make<double>(nb);
            h->xbar = ar.make<double>(3 * nb);
            h->xtil = ar.make<double>(3 * nb);
        } else {
            double* ones = ar.make<double>(nb);
            fill<double>(ones, 1.0, nb, s);
            h->hL = build_hierarchy(Km, ones, 1, o, ar, s, nullptr, true);
            ar.free(ones);
            h->Ls = sell_from_bsr<double>(Km, ar, s);
            h->mslot.h = ctx->c.pinned.get();
            h->mslot.d = PinnedPool::device_ptr(h->mslot.h);
            h->mslot.h[15] = 0.0;
        }
        HIPCHK(hipStreamSynchronize(s));
        h->st.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = h.release();
        return SCR_OK;
    } catch (const std::exception& e) {
        if (h) {
            h->gOuter.reset(); h->gA.reset(); h->gS.reset(); h->gA32.reset();
            (void)hipStreamSynchronize(s);
            if (h->mslot.h) h->ctx->pinned.put(h->mslot.h);
            h->ar.reset();
            (void)hipStreamSynchronize(s);
        }
        return fail(e);
    }
}

scr_status amg_update(scr_handle* h, const scr_bsr* K, const double* coords, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!h || !K) throw Error(SCR_E_INVALID, "NULL argument");
        if (h->broken) throw Error(SCR_E_INVALID, "handle left unusable by a failed amg_update");
        if (!K->row_ptr || !K->col_idx || !K->val) throw Error(SCR_E_INVALID, "NULL matrix array");
        DBsr& Km = h->K;
        if (K->bs != Km.br || K->n_brows != h->nb || K->nnzb != Km.nnzb)
            throw Error(SCR_E_INVALID, "block size, row count or nnzb differ from the handle's matrix");
        HIPCHK(hipSetDevice(h->ctx->device));
        Arena& ar = *h->ar;
        const int64_t nb = h->nb;
        // the pattern must be the stored one: row_ptr first (bounds for the col_idx compare)
        int* flag = ar.make<int>(1);
        zero_dev(flag, sizeof(int), s);
        pattern_diff_k<<<cdiv(nb + 1, 256), 256, 0, s>>>(nb, K->row_ptr, K->col_idx, Km.rp, Km.ci, flag);
        check_launch("pattern_diff");
        int hf = 0;
        HIPCHK(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ar.free(flag);
        if (hf) throw Error(SCR_E_INVALID, "sparsity pattern differs from the one the handle was set up with");
        int bits = validate_bsr(nb, K->bs, K->nnzb, Km.rp, Km.ci, K->val, ar, s);
        if (bits) {
            std::string m = "malformed matrix:";
            if (bits & 16) m += " non-finite-value";
            if (bits & 32) m += " zero-diagonal";
            if (bits & ~48) m += " pattern";
            throw Error(SCR_E_INVALID, m);
        }
        // from here on a failure leaves the handle half-updated
        h->broken = true;
        copy_dev(Km.v, K->val, Km.nnzb * Km.br * Km.bc * sizeof(double), s);
        if (h->kind == SCR_SYSTEM) {
            split_values(Km, h->A, h->G, h->D, h->C, s);
            schur_update(h->A, h->G, h->D, h->C, h->opts.schur_diag, h->dvec, h->Sh, ar, s);
            if (coords) {
                double* xyz = ar.make<double>(nb * 3);
                copy_dev(xyz, coords, nb * 3 * sizeof(double), s);
                rigid_modes(nb, xyz, h->B, ar, s);
                ar.free(xyz);
            }
            update_hierarchy(*h->hA, h->A.v, coords ? h->B : nullptr, ar, s);
            update_hierarchy(*h->hS, h->Sh.v, nullptr, ar, s);
            for (DSell<double>* M : {&h->Ks, &h->As, &h->Gs, &h->Ds, &h->Cs}) sell_free(*M, ar);
            h->Ks = sell_from_bsr<double>(Km, ar, s);
            h->As = sell_from_bsr<double>(h->A, ar, s);
            h->Gs = sell_from_bsr<double>(h->G, ar, s);
            h->Ds = sell_from_bsr<double>(h->D, ar, s);
            h->Cs = sell_from_bsr<double>(h->C, ar, s);
            if (h->Shs.nslices) {
                sell_free(h->Shs, ar);
                h->Shs = sell_from_bsr<double>(h->Sh, ar, s);
            }
        } else {
            update_hierarchy(*h->hL, Km.v, nullptr, ar, s);
            sell_free(h->Ls, ar);
            h->Ls = sell_from_bsr<double>(Km, ar, s);
        }
        HIPCHK(hipStreamSynchronize(s));
        h->broken = false;
        h->st.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return SCR_OK;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        return fail(e);
    }
}

scr_status scr_set_outlets(scr_handle* h, int n_out, const int64_t* off, const int32_t* blk, const double* a,
                           const double* m, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!h) throw Error(SCR_E_INVALID, "NULL handle");
        if (h->kind != SCR_SYSTEM) throw Error(SCR_E_INVALID, "outlets belong to an SCR_SYSTEM handle");
        if (n_out < 0) throw Error(SCR_E_INVALID, "n_out < 0");
        if (n_out > 0 && (!off || !m)) throw Error(SCR_E_INVALID, "NULL off or m");
        HIPCHK(hipSetDevice(h->ctx->device));
        Arena& ar = *h->ar;
        int64_t ne = n_out > 0 ? off[n_out] : 0;
        if (n_out > 0) {
            if (off[0] != 0) throw Error(SCR_E_INVALID, "off[0] != 0");
            for (int k = 0; k < n_out; ++k)
                if (off[k + 1] < off[k]) throw Error(SCR_E_INVALID, "off is not nondecreasing");
            for (int k = 0; k < n_out; ++k)
                if (!std::isfinite(m[k])) throw Error(SCR_E_INVALID, "non-finite coefficient");
            if (ne > 0 && (!blk || !a)) throw Error(SCR_E_INVALID, "NULL blk or a");
        }
        // validate the (small) entry lists on the host before anything is replaced
        std::vector<int32_t> hb(ne);
        std::vector<double> ha(3 * ne);
        if (ne > 0) {
            HIPCHK(hipMemcpyAsync(hb.data(), blk, ne * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(ha.data(), a, 3 * ne * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            std::vector<uint8_t> seen(h->nb, 0);
            for (int64_t e = 0; e < ne; ++e) {
                if (hb[e] < 0 || hb[e] >= h->nb) throw Error(SCR_E_INVALID, "outlet block row out of range");
                if (seen[hb[e]]) throw Error(SCR_E_INVALID, "a block row appears twice in the outlet lists");
                seen[hb[e]] = 1;
            }
            for (double v : ha)
                if (!std::isfinite(v)) throw Error(SCR_E_INVALID, "non-finite outlet vector");
        }
        for (void* p : {(void*)h->out_blk, (void*)h->out_id, (void*)h->out_off, (void*)h->out_a, (void*)h->out_m,
                        (void*)h->out_s})
            ar.free(p);
        h->out_blk = h->out_id = nullptr;
        h->out_off = nullptr;
        h->out_a = h->out_m = h->out_s = nullptr;
        h->n_out = 0;
        h->n_oe = 0;
        if (n_out == 0) return SCR_OK;
        std::vector<int32_t> hid(ne);
        for (int k = 0; k < n_out; ++k)
            for (int64_t e = off[k]; e < off[k + 1]; ++e) hid[e] = k;
        h->out_off = ar.make<int64_t>(n_out + 1);
        h->out_m = ar.make<double>(n_out);
        h->out_s = ar.make<double>(n_out);
        h->out_blk = ar.make<int32_t>(ne > 0 ? ne : 1);
        h->out_id = ar.make<int32_t>(ne > 0 ? ne : 1);
        h->out_a = ar.make<double>(3 * (ne > 0 ? ne : 1));
        HIPCHK(hipMemcpyAsync(h->out_off, off, (n_out + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(h->out_m, m, n_out * sizeof(double), hipMemcpyHostToDevice, s));
        if (ne > 0) {
            HIPCHK(hipMemcpyAsync(h->out_blk, hb.data(), ne * sizeof(int32_t), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(h->out_id, hid.data(), ne * sizeof(int32_t), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(h->out_a, ha.data(), 3 * ne * sizeof(double), hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        h->n_out = n_out;
        h->n_oe = ne;
        return SCR_OK;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        return fail(e);
    }
}

scr_status scr_handle_destroy(scr_handle* h) {
    if (!h) return SCR_OK;
    try {
        hipStream_t s = h->ar ? h->ar->stream() : nullptr;
        h->gOuter.reset(); h->gA.reset(); h->gS.reset(); h->gA32.reset();
        h->hA.reset(); h->hS.reset(); h->hL.reset();
        (void)hipStreamSynchronize(s);
        if (h->mslot.h) h->ctx->pinned.put(h->mslot.h);
        h->ar.reset();
        (void)hipStreamSynchronize(s);
        delete h;
        return SCR_OK;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

int64_t scr_handle_bytes(const scr_handle* h) { return (h && h->ar) ? h->ar->bytes() : 0; }
int64_t scr_handle_peak_bytes(const scr_handle* h) { return (h && h->ar) ? h->ar->peak() : 0; }

scr_status scr_solve(scr_handle* h, const double* b, double* x, const scr_solve_opts* opts, void* stream,
                     scr_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!h || !b || !x) throw Error(SCR_E_INVALID, "NULL argument");
        if (h->kind != SCR_SYSTEM) throw Error(SCR_E_INVALID, "scr_solve needs an SCR_SYSTEM handle");
        if (h->broken) throw Error(SCR_E_INVALID, "handle left unusable by a failed amg_update");
        HIPCHK(hipSetDevice(h->ctx->device));
        scr_solve_opts o;
        if (opts) o = *opts;
        else scr_default_solve_opts(&o);
        check_opts(o);
        ensure_workspaces(h, o, s);
        double setup_ms = h->st.t_setup_ms;
        h->st = scr_stats{};
        h->st.t_setup_ms = setup_ms;
        h->so = o;
        const int64_t nb = h->nb;
        interleaved_to_split(nb, b, h->bs, s);
        if (o.use_x0) interleaved_to_split(nb, x, h->xs, s);
        KOp kop(h);
        ScrPrec prec_scr(h);
        SimplePrec prec_simple(h);
        if (o.precond == SCR_PRECOND_SIMPLE) ensure_simple(h, s);
        Op& prec = o.precond == SCR_PRECOND_SIMPLE ? static_cast<Op&>(prec_simple) : static_cast<Op&>(prec_scr);
        KStat k = h->gOuter->solve(kop, prec, h->bs, h->xs, o.tol, o.max_it, o.use_x0 != 0, true, s);
        split_to_interleaved(nb, h->xs, x, s);
        HIPCHK(hipStreamSynchronize(s));
        h->ctx->prof.harvest();
        h->st.outer_it = (int)k.iters;
        h->st.rel_res_true = k.rel_res;
        h->st.converged = k.converged ? 1 : 0;
        h->st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        h->st.device_bytes = h->ar->bytes();
        if (stats) *stats = h->st;
        return k.converged ? SCR_OK : SCR_NOT_CONVERGED;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        if (stats && h) *stats = h->st;
        return fail(e);
    }
}

scr_status mesh_motion_solve(scr_handle* h, const double* b, double* x, const scr_solve_opts* opts, void* stream,
                             scr_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!h || !b || !x) throw Error(SCR_E_INVALID, "NULL argument");
        if (h->kind != MESH_SYSTEM) throw Error(SCR_E_INVALID, "mesh_motion_solve needs a MESH_SYSTEM handle");
        if (h->broken) throw Error(SCR_E_INVALID, "handle left unusable by a failed amg_update");
        HIPCHK(hipSetDevice(h->ctx->device));
        scr_solve_opts o;
        if (opts) o = *opts;
        else scr_default_solve_opts(&o);
        check_opts(o);
        ensure_workspaces(h, o, s);
        double setup_ms = h->st.t_setup_ms;
        h->st = scr_stats{};
        h->st.t_setup_ms = setup_ms;
        bool ok = mesh_solve_run(h, b, x, o, h->mws, s);
        HIPCHK(hipStreamSynchronize(s));
        h->st.converged = ok ? 1 : 0;
        h->st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        h->st.device_bytes = h->ar->bytes();
        if (stats) *stats = h->st;
        return ok ? SCR_OK : SCR_NOT_CONVERGED;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        if (stats && h) *stats = h->st;
        return fail(e);
    }
}

scr_status mesh_motion_solve_noalloc(scr_handle* h, const double* b, double* x, const scr_solve_opts* opts,
                                     void* stream, scr_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!h || !b || !x) throw Error(SCR_E_INVALID, "NULL argument");
        if (h->kind != MESH_SYSTEM) throw Error(SCR_E_INVALID, "mesh_motion_solve_noalloc needs a MESH_SYSTEM handle");
        if (h->broken) throw Error(SCR_E_INVALID, "handle left unusable by a failed amg_update");
        const int64_t need = Pcg3::workspace_doubles(h->nb);
        if (need > NOALLOC_SCRATCH_DOUBLES)
            throw Error(SCR_E_INVALID, "mesh of " + std::to_string(h->nb) + " nodes needs " +
                                           std::to_string(need * 8) + " bytes of scratch; the static scratch holds " +
                                           std::to_string(NOALLOC_SCRATCH_DOUBLES * 8));
        HIPCHK(hipSetDevice(h->ctx->device));
        double* ws = noalloc_scratch(h->ctx->device);
        scr_solve_opts o;
        if (opts) o = *opts;
        else scr_default_solve_opts(&o);
        check_opts(o);
        double setup_ms = h->st.t_setup_ms;
        h->st = scr_stats{};
        h->st.t_setup_ms = setup_ms;
        bool ok = mesh_solve_run(h, b, x, o, ws, s);
        HIPCHK(hipStreamSynchronize(s));
        h->st.converged = ok ? 1 : 0;
        h->st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        h->st.device_bytes = h->ar->bytes();
        if (stats) *stats = h->st;
        return ok ? SCR_OK : SCR_NOT_CONVERGED;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        if (stats && h) *stats = h->st;
        return fail(e);
    }
}

int64_t scr_footprint_estimate(int kind, int64_t n_brows, int64_t nnzb, const scr_amg_opts* amg,
                               const scr_solve_opts* solve) {
    scr_solve_opts so;
    if (solve) so = *solve;
    else scr_default_solve_opts(&so);
    const double pad = 1.15;     // sliced-ELL padding
    const double amgf = (amg && amg->precision != SCR_FP64) ? 0.5 : 1.0;
    double bytes;
    if (kind == SCR_SYSTEM) {
        double perblk = 132.0 + (76.0 + 28.0 + 28.0 + 12.0)          // K and its split (FP64 + indices)
                        + pad * (132.0 + 76.0 + 28.0 + 28.0 + 12.0)  // solve-phase copies
                        + 5.0 * 12.0 * 2.0;                          // S^ (about 5 entries per K block) and its copy
        double hier = 3.0 * nnzb * (76.0 * 1.8 * (1.0 + amgf)) + 5.0 * nnzb * 12.0 * 2.0 * (1.0 + amgf);
        double krylov = 8.0 * n_brows * (4.0 * (2 * so.restart + 1) + 3.0 * (2 * so.restart_inner + 1) +
                                         1.0 * (2 * so.restart_inner + 1) + 24.0);
        bytes = perblk * nnzb + hier + krylov + 64.0 * 1024 * 1024 + 8.0 * 1024 * 1024 * 2;
    } else {
        // L and its solve copy; the hierarchy (values in FP64 for setup, T for the V-cycle); one- and
        // three-column level vectors (28 per level, the levels adding up to about 1.1 n); the CG
        // workspace (15 n)
        double hier = nnzb * 12.0 * 3.0 * (1.0 + amgf);
        double vecs = 8.0 * n_brows * (1.1 * 28.0 * (amgf < 1.0 ? 0.5 : 1.0) + 1.1 * 2.0 + 15.0 + 12.0);
        bytes = nnzb * 12.0 * (1.0 + pad) + hier + vecs + 16.0 * 1024 * 1024;
    }
    return (int64_t)bytes;
}

// ---------------------------------------------------------------- inspection
static Hierarchy* which_hier(scr_handle* h, int which) {
    Hierarchy* H = which == 0 ? h->hA.get() : which == 1 ? h->hS.get() : which == 2 ? h->hL.get() : nullptr;
    if (!H) throw Error(SCR_E_INVALID, "no such hierarchy on this handle");
    return H;
}

scr_status scr_hier_levels(scr_handle* h, int which, int* nlev) {
    try {
        if (!h || !nlev) throw Error(SCR_E_INVALID, "NULL argument");
        *nlev = (int)which_hier(h, which)->L.size();
        return SCR_OK;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

scr_status scr_hier_level_info(scr_handle* h, int which, int level, int64_t* info, double* lam) {
    try {
        if (!h || !info || !lam) throw Error(SCR_E_INVALID, "NULL argument");
        Hierarchy* H = which_hier(h, which);
        if (level < 0 || level >= (int)H->L.size()) throw Error(SCR_E_INVALID, "level out of range");
        LevelSetup& L = H->L[level];
        info[0] = L.A.nr; info[1] = L.b; info[2] = L.k; info[3] = L.A.nnzb; info[4] = L.nagg;
        info[5] = L.P.nnzb; info[6] = L.R.nnzb; info[7] = H->ncoarse;
        *lam = L.lam;
        return SCR_OK;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

scr_status scr_hier_level_copy(scr_handle* h, int which, int level, int field, void* dst) {
    try {
        if (!h || !dst) throw Error(SCR_E_INVALID, "NULL argument");
        HIPCHK(hipSetDevice(h->ctx->device));
        Hierarchy* H = which_hier(h, which);
        if (level < 0 || level >= (int)H->L.size()) throw Error(SCR_E_INVALID, "level out of range");
        LevelSetup& L = H->L[level];
        const void* src = nullptr;
        size_t bytes = 0;
        auto mat = [&](const DBsr& M, int f) {
            if (!M.rp) throw Error(SCR_E_INVALID, "level has no such matrix");
            if (f == 0) { src = M.rp; bytes = (M.nr + 1) * sizeof(int32_t); }
            else if (f == 1) { src = M.ci; bytes = M.nnzb * sizeof(int32_t); }
            else { src = M.v; bytes = M.nnzb * M.br * M.bc * sizeof(double); }
        };
        switch (field) {
            case 0: case 1: case 2: mat(L.A, field); break;
            case 3: src = L.agg; bytes = L.A.nr * sizeof(int32_t); break;
            case 4: case 5: case 6: mat(L.P, field - 4); break;
            case 7: case 8: case 9: mat(L.R, field - 7); break;
            case 10: src = L.strong; bytes = L.A.nnzb; break;
            case 11: src = L.dead; bytes = L.nagg * L.k; break;
            case 12: src = L.Dinv; bytes = L.A.nr * L.b * L.b * sizeof(double); break;
            case 13: src = L.B; bytes = L.A.nr * L.b * L.k * sizeof(double); break;
            case 15: src = L.func; bytes = L.A.nr; break;
            default: throw Error(SCR_E_INVALID, "unknown field");
        }
        if (!src) throw Error(SCR_E_INVALID, "field not present on this level");
        if (bytes) HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        return SCR_OK;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

scr_status scr_matrix_copy(scr_handle* h, int which, int field, void* dst, int64_t* info) {
    try {
        if (!h || !info) throw Error(SCR_E_INVALID, "NULL argument");
        if (h->kind != SCR_SYSTEM) throw Error(SCR_E_INVALID, "not an SCR_SYSTEM handle");
        HIPCHK(hipSetDevice(h->ctx->device));
        const DBsr* M = which == 0 ? &h->A : which == 1 ? &h->G : which == 2 ? &h->D : which == 3 ? &h->C
                        : which == 4 ? &h->Sh : nullptr;
        if (!M) throw Error(SCR_E_INVALID, "unknown matrix");
        info[0] = M->nr; info[1] = M->nnzb; info[2] = M->br; info[3] = M->bc;
        if (!dst) return SCR_OK;
        if (field == 0) HIPCHK(hipMemcpy(dst, M->rp, (M->nr + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        else if (field == 1) HIPCHK(hipMemcpy(dst, M->ci, M->nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
        else HIPCHK(hipMemcpy(dst, M->v, M->nnzb * M->br * M->bc * sizeof(double), hipMemcpyDeviceToHost));
        return SCR_OK;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

scr_status scr_apply(scr_handle* h, int op, const double* x, double* y, const scr_solve_opts* opts, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    try {
        if (!h || !x || !y) throw Error(SCR_E_INVALID, "NULL argument");
        HIPCHK(hipSetDevice(h->ctx->device));
        scr_solve_opts o;
        if (opts) o = *opts;
        else scr_default_solve_opts(&o);
        check_opts(o);
        ensure_workspaces(h, o, s);
        h->so = o;
        bool scr = h->kind == SCR_SYSTEM;
        if ((op <= 9 || op == 12 || op == 13) != scr)
            throw Error(SCR_E_INVALID, "operator not available on this handle kind");
        switch (op) {
            case 0: { KOp k(h); k.apply(x, y, s); break; }
            case 1: { AOp a(h); a.apply(x, y, s); break; }
            case 2: h->hA->vcycle(x, y, s); break;
            case 3: h->hS->vcycle(x, y, s); break;
            case 4: { SchurOp so(h); so.apply(x, y, s); break; }
            case 5: { ScrPrec p(h); p.apply(x, y, s); break; }
            case 6: sell_mv<double>(h->Gs, x, nullptr, y, 0, s); break;
            case 7: sell_mv<double>(h->Ds, x, nullptr, y, 0, s); break;
            case 8: sell_mv<double>(h->Cs, x, nullptr, y, 0, s); break;
            case 9: {
                DSell<double> S = sell_from_bsr<double>(h->Sh, *h->ar, s);
                sell_mv<double>(S, x, nullptr, y, 0, s);
                HIPCHK(hipStreamSynchronize(s));
                sell_free(S, *h->ar);
                break;
            }
            case 10: sell_mv<double>(h->Ls, x, nullptr, y, 0, s); break;
            case 11: h->hL->vcycle(x, y, s); break;
            case 12: { ensure_simple(h, s); SimplePrec p(h); p.apply(x, y, s); break; }
            case 13: copy_d(3 * h->nb, h->dvec, y, s); break;
            default: throw Error(SCR_E_INVALID, "unknown operator");
        }
        HIPCHK(hipStreamSynchronize(s));
        return SCR_OK;
    } catch (const std::exception& e) {
        (void)hipStreamSynchronize(s);
        return fail(e);
    }
}

}  // extern "C"
