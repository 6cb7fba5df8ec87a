// solver.h -- Krylov drivers (krylov.hip), AMG hierarchies (amg.hip) and the handle (scr.hip).
#pragma once
#include <memory>

#include "kernels.h"

namespace scr {

// A linear operator or preconditioner on device vectors of T (FP64, or FP32 for the mixed
// precision inner solves).
template <typename T>
struct OpT {
    virtual void apply(const T* x, T* y, hipStream_t s) = 0;
    virtual ~OpT() = default;
};
using Op = OpT<double>;

struct KStat {
    int64_t iters = 0;
    double rel_res = 0.0;
    bool converged = false;
};

// Deterministic FP64 reductions: a fixed grid per vector length, per-block partials summed in a
// fixed order by a one-block kernel.
struct Reducer {
    int64_t n = 0;
    int grid = 0;
    double* partials = nullptr;      // grid * 64
    double* out = nullptr;           // 64 results
    void init(int64_t n_, Arena& ar, hipStream_t s);
    void release(Arena& ar) {
        ar.free(partials); ar.free(out);
        partials = nullptr; out = nullptr;
    }
};

// Host side of a published status slot: spin until the sequence number arrives (the stream is
// polled so that a failed launch surfaces as an error instead of a wait forever).
struct StatusSlot {
    double* h = nullptr;       // host address (pinned, mapped)
    double* d = nullptr;       // device address of the same slot
    double seq = 0.0;
    double next() { return seq += 1.0; }
    void wait(hipStream_t s) const;
};

// Right-preconditioned flexible GMRES(m) (Saad 1993) with CGS2 Arnoldi; the Hessenberg matrix,
// Givens rotations and least-squares solve stay in device memory (FP64); the host reads one
// residual estimate per iteration.  The Krylov vectors are T; every dot product and vector update
// is computed in FP64 and rounded to T when stored.
template <typename T>
class GmresT {
   public:
    GmresT(int64_t n, int m, Arena& ar, hipStream_t s);
    ~GmresT();
    KStat solve(OpT<T>& A, OpT<T>& M, const T* b, T* x, double tol, int maxit, bool use_x0, bool check_true,
                hipStream_t s);
    int64_t n() const { return n_; }

   private:
    int64_t n_;
    int m_;
    Arena* ar_;
    T *V_, *Z_;
    double* st_;
    Reducer red_;
    StatusSlot slot_;
};
using Gmres = GmresT<double>;

// Preconditioned CG, or flexible CG with the Polak-Ribiere beta (Notay 2000), on three
// node-interleaved columns at once (the mesh-motion system of Sec. 5.2.2: one Laplacian for x, y
// and z): one product with L and one V-cycle of AMG(L) per iteration for all three, each column
// with its own recurrence scalars and its own stopping test.  Per column the arithmetic and the
// reduction order are those of a one-column CG with the same grid.
// The workspace (Pcg3::workspace_doubles(n) doubles) and the status slot are the caller's (the
// slot's sequence number must persist from one solve to the next).
class Pcg3 {
   public:
    static int64_t workspace_doubles(int64_t n);
    Pcg3(int64_t n, double* ws, StatusSlot* slot);
    struct Result {
        int64_t iters[3] = {0, 0, 0};
        double rel[3] = {0.0, 0.0, 0.0};
        bool converged[3] = {false, false, false};
    };
    // x (3n, interleaved) is overwritten; A and M act on interleaved three-column vectors
    Result solve(Op& A, Op& M, const double* b, double* x, double tol, int maxit, bool flexible, hipStream_t s);

   private:
    int64_t n_;
    int grid_;
    double *r_, *z_, *p_, *q_, *rold_, *st_, *part_, *out_;
    StatusSlot* slot_;
};

template <typename T>
double device_norm(const T* x, int64_t n, Reducer& red, StatusSlot& slot, hipStream_t s);

// ---------------------------------------------------------------- AMG (amg.hip)
struct LevelSetup {
    DBsr A, P, R;
    int b = 0, k = 0;
    int64_t nagg = 0;
    int32_t* agg = nullptr;
    uint8_t* strong = nullptr;
    uint8_t* dead = nullptr;
    double* Dinv = nullptr;
    double* B = nullptr;
    uint8_t* func = nullptr;         // classical AMG: the function (unknown) of each scalar row
    double* ell = nullptr;           // classical AMG, l1 smoother: the l1 term of each row's diagonal
    double lam = 0.0;
    // kept for the numeric re-setup: aggregate member lists and the pattern of A P (no values)
    int32_t *mrp = nullptr, *mem = nullptr;
    DBsr AP;
};

class Hierarchy {
   public:
    virtual ~Hierarchy() = default;
    // y = V-cycle(x), zero initial guess; FP64 in and out (cast at the boundary in MIXED).
    virtual void vcycle(const double* x, double* y, hipStream_t s) = 0;
    // rebuild the solve-phase copies (sliced ELL in T, D^-1, smoothing coefficients) from L
    virtual void refresh(Arena& ar, hipStream_t s) = 0;
    // FP32 hierarchies: the V-cycle on FP32 vectors (no conversions), and the FP32 sliced-ELL copy
    // of the level-0 matrix (nullptr when the hierarchy is FP64 or has a single level)
    virtual void vcycle_f(const float* x, float* y, hipStream_t s) = 0;
    // scalar hierarchies built with `three`: the V-cycle on three node-interleaved columns (the mesh
    // Laplacian acts on x, y and z alike), FP64 in and out; counts three V-cycles
    virtual void vcycle3(const double* x, double* y, hipStream_t s) = 0;
    bool three = false;
    virtual const DSell<float>* level0_f() const = 0;
    std::vector<LevelSetup> L;
    double* cinv = nullptr;          // dense inverse of the coarsest matrix (FP64)
    int64_t ncoarse = 0;
    double coarse_eta = 0.0;         // backward error of one solve with cinv (accuracy check)
    bool coarse_pivoted = false;     // cinv came from the partial-pivoting fallback
    scr_amg_opts opts{};
    int64_t vcycles = 0;
    int64_t n0() const { return L.empty() ? 0 : L[0].A.nr * L[0].b; }
};

// prof: the context profiler, or nullptr; when set, level-0 smoother steps are timed.
std::unique_ptr<Hierarchy> build_hierarchy(const DBsr& A0, const double* B0, int k, const scr_amg_opts& o, Arena& ar,
                                           hipStream_t s, Profiler* prof = nullptr, bool three = false);

// Numeric re-setup for new level-0 values on the same pattern (and, if B0 is not NULL, a new
// near-null space): aggregates and every pattern are kept, every value-dependent quantity of every
// level is recomputed as in build_hierarchy.
void update_hierarchy(Hierarchy& H, const double* vals0, const double* B0, Arena& ar, hipStream_t s);

// new values of S^ = C - D d^-1 G into its existing pattern (the patterns of A, G, D, C unchanged)
void schur_update(const DBsr& A, const DBsr& G, const DBsr& D, const DBsr& C, int mode, double* d, DBsr& S, Arena& ar,
                  hipStream_t s);

// values of the split of K into A, G, D, C (patterns already set up by split_blocks)
void split_values(const DBsr& K, DBsr& A, DBsr& G, DBsr& D, DBsr& C, hipStream_t s);

// classical AMG (classical.hip): the hierarchy of Sec. 5.2's settings for A0 (scalar, or b x b
// blocks taken as b functions), and its set-up again for new level-0 values
std::unique_ptr<Hierarchy> build_classical(const DBsr& A0, const scr_amg_opts& o, Arena& ar, hipStream_t s,
                                           bool three);
void update_classical(Hierarchy& H, const double* vals0, Arena& ar, hipStream_t s);

// building blocks shared by the two AMG set-ups (amg.hip)
DBsr bsr_alloc(int64_t nr, int64_t nc, int br, int bc, int64_t nnzb, Arena& ar);
void bsr_release(DBsr& M, Arena& ar);
// C = X Y on the structural pattern (rows with rowmask[i] == 0 left empty when rowmask is given);
// each entry sums its products in the order of X's row
DBsr spgemm(const DBsr& X, const DBsr& Y, const uint8_t* rowmask, Arena& ar, hipStream_t s);
DBsr transpose(const DBsr& M, Arena& ar, hipStream_t s);
// D^-1 and lambda_hat of a level (err, lamd: one-element device scratch)
void level_diag(LevelSetup& L, int l, int* err, unsigned long long* lamd, hipStream_t s);
// explicit inverse of the coarsest level into H.cinv (fast, with a pivoted fallback)
void coarse_inverse(Hierarchy& H, int* err, Arena& ar, hipStream_t s);

// rigid-body modes (6 columns) of nb nodes from coordinates, shifted by their mean
void rigid_modes(int64_t nb, const double* xyz, double* B, Arena& ar, hipStream_t s);

// split K (4x4) into A (3x3), G (3x1), D (1x3), C (1x1) and build S^ = C - D diag(A)^-1 G
void split_blocks(const DBsr& K, DBsr& A, DBsr& G, DBsr& D, DBsr& C, Arena& ar, hipStream_t s);
// S^ = C - D d^-1 G; d (3n, written) = diag(A) (mode 0) or the absolute row sums of A (mode 1)
DBsr schur_approx(const DBsr& A, const DBsr& G, const DBsr& D, const DBsr& C, int mode, double* d, Arena& ar,
                  hipStream_t s);

}  // namespace scr
