// krylov.hip -- FP64 vector kernels, deterministic reductions and the Krylov drivers:
// flexible GMRES with classical Gram-Schmidt applied twice (CGS2) and device-resident Givens
// rotations, and (flexible) preconditioned CG on three interleaved columns.  Every reduction uses a grid fixed by the
// vector length and sums per-block partials in block order, so results are bitwise
// reproducible run to run.
#include <immintrin.h>

#include <cmath>

#include "solver.h"

namespace scr {

constexpr int RTPB = 256;
constexpr int RMAXJ = 64;   // partial slots per block

// ------------------------------------------------------------------ vector kernels
__global__ void axpby_k(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
    if (n > 0) axpby_k<<<cdiv(n, 256), 256, 0, s>>>(n, a, x, b, y);
    check_launch("axpby");
}
void copy_d(int64_t n, const double* x, double* y, hipStream_t s) {
    if (n > 0) copy_dev(y, x, n * sizeof(double), s);
}

__global__ void i2s_k(int64_t nb, const double* __restrict__ a, double* __restrict__ sv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    sv[3 * i] = a[4 * i]; sv[3 * i + 1] = a[4 * i + 1]; sv[3 * i + 2] = a[4 * i + 2];
    sv[3 * nb + i] = a[4 * i + 3];
}
__global__ void s2i_k(int64_t nb, const double* __restrict__ sv, double* __restrict__ a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    a[4 * i] = sv[3 * i]; a[4 * i + 1] = sv[3 * i + 1]; a[4 * i + 2] = sv[3 * i + 2];
    a[4 * i + 3] = sv[3 * nb + i];
}
void interleaved_to_split(int64_t nb, const double* a, double* sv, hipStream_t s) {
    if (nb > 0) i2s_k<<<cdiv(nb, 256), 256, 0, s>>>(nb, a, sv);
    check_launch("i2s");
}
void split_to_interleaved(int64_t nb, const double* sv, double* a, hipStream_t s) {
    if (nb > 0) s2i_k<<<cdiv(nb, 256), 256, 0, s>>>(nb, sv, a);
    check_launch("s2i");
}
// ------------------------------------------------------------------ reduction machinery
void Reducer::init(int64_t n_, Arena& ar, hipStream_t s) {
    n = n_;
    int64_t g = cdiv(n, 4 * RTPB);
    grid = (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
    partials = ar.make<double>((size_t)grid * RMAXJ);
    out = ar.make<double>(RMAXJ);
}

template <int J>
__device__ __forceinline__ void block_partials(const double (&acc)[J], int jn, double* __restrict__ partials) {
    __shared__ double red[RTPB / WAVE][J];
    int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int j = 0; j < J; ++j)
        if (j < jn) {
            double v = wave_sum(acc[j]);
            if (lane == 0) red[w][j] = v;
        }
    __syncthreads();
    for (int j = threadIdx.x; j < jn; j += RTPB) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < RTPB / WAVE; ++q) t += red[q][j];
        partials[(int64_t)blockIdx.x * RMAXJ + j] = t;
    }
}

// Final sum of the per-block partials (j < jn) by one block launched after the partials kernel:
// thread t adds blocks t, t + 256, ... in order, then a fixed shuffle/LDS tree.  Deterministic
// for a fixed grid; the kernel boundary makes every block's partials visible (no fences).
template <int J>
__device__ __forceinline__ void final_sums(const double* __restrict__ partials, int nblk, int jn,
                                           double* __restrict__ out) {
    __shared__ double red[RTPB / WAVE][J];
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RTPB) {
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < jn) acc[j] += partials[(int64_t)b * RMAXJ + j];
    }
    int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int j = 0; j < J; ++j)
        if (j < jn) {
            double v = wave_sum(acc[j]);
            if (lane == 0) red[w][j] = v;
        }
    __syncthreads();
    for (int j = threadIdx.x; j < jn; j += RTPB) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < RTPB / WAVE; ++q) t += red[q][j];
        out[j] = t;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ plain dot (FP64 accumulation)
template <typename T>
__global__ void __launch_bounds__(RTPB) dot_part_k(int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                                                   double* __restrict__ partials) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * RTPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTPB)
        acc[0] += (double)x[i] * (double)y[i];
    block_partials<1>(acc, 1, partials);
}
// y = a x + b y in FP64, rounded to T
template <typename T>
__global__ void axpby_t_k(int64_t n, double a, const T* __restrict__ x, double b, T* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (T)(a * (double)x[i] + b * (double)y[i]);
}
template <int J>
__global__ void __launch_bounds__(RTPB) sum_k(const double* __restrict__ partials, int nblk, int jn, double* __restrict__ out) {
    final_sums<J>(partials, nblk, jn, out);
}

// thread 0 of a finishing kernel: copy n status values to the host slot, then the sequence
// number (system-scope fence in between, so the host never sees the number before the values)
__device__ __forceinline__ void publish(double* __restrict__ hslot, const double* __restrict__ vals, int n, double seq) {
    for (int i = 0; i < n; ++i) hslot[i] = vals[i];
    __threadfence_system();
    *(volatile double*)(hslot + 15) = seq;
}

void StatusSlot::wait(hipStream_t s) const {
    volatile double* flag = h + 15;
    for (uint64_t it = 0;; ++it) {
        if (*flag == seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return;
        }
        if ((it & 4095) == 4095) {
            hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (*flag == seq) continue;
                throw Error(SCR_E_HIP, "Krylov status was not published");
            }
            if (e != hipErrorNotReady) throw Error(SCR_E_HIP, std::string("stream error: ") + hipGetErrorString(e));
        }
        _mm_pause();
    }
}

__global__ void __launch_bounds__(RTPB) sum_pub_k(const double* __restrict__ partials, int nblk, double* __restrict__ out,
                                                  double* __restrict__ hslot, double seq) {
    final_sums<1>(partials, nblk, 1, out);
    if (threadIdx.x == 0) publish(hslot, out, 1, seq);
}

template <typename T>
double device_norm(const T* x, int64_t n, Reducer& red, StatusSlot& slot, hipStream_t s) {
    dot_part_k<<<red.grid, RTPB, 0, s>>>(n, x, x, red.partials);
    sum_pub_k<<<1, RTPB, 0, s>>>(red.partials, red.grid, red.out, slot.d, slot.next());
    check_launch("dot");
    slot.wait(s);
    return std::sqrt(slot.h[0]);
}
template double device_norm<double>(const double*, int64_t, Reducer&, StatusSlot&, hipStream_t);
template double device_norm<float>(const float*, int64_t, Reducer&, StatusSlot&, hipStream_t);

// ------------------------------------------------------------------ GMRES kernels
// state layout (doubles): H[(m+1)*m] | cs[m] | sn[m] | g[m+1] | y[m] | h1[64] | h2[64] | scal[8]
struct GLay {
    int m;
    __host__ __device__ int H() const { return 0; }
    __host__ __device__ int cs() const { return (m + 1) * m; }
    __host__ __device__ int sn() const { return cs() + m; }
    __host__ __device__ int g() const { return sn() + m; }
    __host__ __device__ int y() const { return g() + m + 1; }
    __host__ __device__ int h1() const { return y() + m; }
    __host__ __device__ int h2() const { return h1() + 64; }
    __host__ __device__ int scal() const { return h2() + 64; }
    __host__ __device__ int size() const { return scal() + 8; }
};
enum { S_BETA = 0, S_EST = 1, S_HN = 2, S_INV = 3, S_FLAG = 4 };

// beta = ||v|| (from the partials of v.v); g = [beta, 0, ...]; inv = 1/beta
__global__ void __launch_bounds__(RTPB) gm_init_fin_k(const double* __restrict__ partials, int nblk,
                                                      double* __restrict__ st, int m, double* __restrict__ hslot,
                                                      double seq) {
    GLay L{m};
    double* sc = st + L.scal();
    final_sums<1>(partials, nblk, 1, sc + S_HN);
    if (threadIdx.x == 0) {
        double beta = sqrt(sc[S_HN]);
        sc[S_BETA] = beta;
        sc[S_EST] = beta;
        sc[S_INV] = beta > 0.0 ? 1.0 / beta : 0.0;
        sc[S_FLAG] = isfinite(beta) ? 0.0 : 1.0;
        double* g = st + L.g();
        g[0] = beta;
        for (int i = 1; i <= m; ++i) g[i] = 0.0;
        publish(hslot, sc, 8, seq);
    }
}

template <typename T>
__global__ void scale_by_k(int64_t n, T* __restrict__ v, const double* __restrict__ s) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double f = *s;
    if (i < n) v[i] = (T)((double)v[i] * f);
}

// partials of V_i . w  (i < jn)
template <int J, typename T>
__global__ void __launch_bounds__(RTPB) mdot_k(int64_t n, int jn, const T* __restrict__ V, int64_t ld,
                                               const T* __restrict__ w, double* __restrict__ partials) {
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * RTPB) {
        double we = w[e];
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < jn) acc[j] += (double)V[j * ld + e] * we;
    }
    block_partials<J>(acc, jn, partials);
}

// w -= sum_i h_i V_i ;  partials of V_i . w
template <int J, typename T>
__global__ void __launch_bounds__(RTPB) upd_dot_k(int64_t n, int jn, const T* __restrict__ V, int64_t ld,
                                                  T* __restrict__ w, const double* __restrict__ h,
                                                  double* __restrict__ partials) {
    __shared__ double hs[J];
    for (int j = threadIdx.x; j < jn; j += RTPB) hs[j] = h[j];
    __syncthreads();
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * RTPB) {
        double v[J];
        double we = w[e];
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < jn) {
                v[j] = V[j * ld + e];
                we -= hs[j] * v[j];
            }
        const T wr = (T)we;     // the stored value enters the dot products
        w[e] = wr;
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < jn) acc[j] += v[j] * (double)wr;
    }
    block_partials<J>(acc, jn, partials);
}

// w -= sum_i h2_i V_i ; partials of ||w||^2
template <int J, typename T>
__global__ void __launch_bounds__(RTPB) upd_norm_k(int64_t n, int jn, const T* __restrict__ V, int64_t ld,
                                                   T* __restrict__ w, const double* __restrict__ h2,
                                                   double* __restrict__ partials) {
    __shared__ double hs[J];
    for (int t = threadIdx.x; t < jn; t += RTPB) hs[t] = h2[t];
    __syncthreads();
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * RTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * RTPB) {
        double we = w[e];
#pragma unroll
        for (int t = 0; t < J; ++t)
            if (t < jn) we -= hs[t] * (double)V[t * ld + e];
        const T wr = (T)we;
        w[e] = wr;
        acc[0] += (double)wr * (double)wr;
    }
    block_partials<1>(acc, 1, partials);
}

// Arnoldi column j (one block): ||w||, H[:,j] = h1 + h2, H[j+1,j] = ||w||, previous rotations,
// new rotation, g update, estimate |g[j+1]|, 1/||w|| for the normalisation.
__global__ void __launch_bounds__(RTPB) arnoldi_fin_k(const double* __restrict__ partials, int nblk,
                                                      double* __restrict__ st, int m, int j, double* __restrict__ hslot,
                                                      double seq) {
    GLay L{m};
    double* sc = st + L.scal();
    final_sums<1>(partials, nblk, 1, sc + S_HN);
    if (threadIdx.x != 0) return;
    double* H = st + L.H();
    double* cs = st + L.cs();
    double* sn = st + L.sn();
    double* g = st + L.g();
    const double* h1 = st + L.h1();
    const double* h2 = st + L.h2();
    double hn = sqrt(sc[S_HN]);
    for (int i = 0; i <= j; ++i) H[i * m + j] = h1[i] + h2[i];
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        double a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
    }
    double a = H[j * m + j], c = H[(j + 1) * m + j];
    double rr = sqrt(a * a + c * c);
    cs[j] = rr == 0.0 ? 1.0 : a / rr;
    sn[j] = rr == 0.0 ? 0.0 : c / rr;
    H[j * m + j] = rr;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    sc[S_HN] = hn;
    sc[S_EST] = fabs(g[j + 1]);
    sc[S_INV] = hn > 0.0 ? 1.0 / hn : 0.0;
    sc[S_FLAG] = (isfinite(hn) && isfinite(sc[S_EST]) && isfinite(rr)) ? 0.0 : 1.0;
    publish(hslot, sc, 8, seq);
}

// back substitution of the j x j upper triangle: y = R^-1 g
__global__ void ysolve_k(double* __restrict__ st, int m, int j) {
    GLay L{m};
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double* H = st + L.H();
    const double* g = st + L.g();
    double* y = st + L.y();
    for (int i = j - 1; i >= 0; --i) {
        double s = g[i];
        for (int t = i + 1; t < j; ++t) s -= H[i * m + t] * y[t];
        y[i] = s / H[i * m + i];
    }
}

// x += sum_i y_i Z_i
template <typename T>
__global__ void __launch_bounds__(RTPB) maxpy_k(int64_t n, int jn, const T* __restrict__ Z, int64_t ld,
                                                const double* __restrict__ y, T* __restrict__ x) {
    __shared__ double ys[RMAXJ];
    for (int j = threadIdx.x; j < jn; j += RTPB) ys[j] = y[j];
    __syncthreads();
    int64_t e = (int64_t)blockIdx.x * RTPB + threadIdx.x;
    if (e >= n) return;
    double xe = x[e];
    for (int j = 0; j < jn; ++j) xe += ys[j] * (double)Z[j * ld + e];
    x[e] = (T)xe;
}

#define JDISPATCH(jn, KERNEL, ...)                                         \
    do {                                                                   \
        if ((jn) <= 4) KERNEL<4>__VA_ARGS__;                               \
        else if ((jn) <= 8) KERNEL<8>__VA_ARGS__;                          \
        else if ((jn) <= 16) KERNEL<16>__VA_ARGS__;                        \
        else if ((jn) <= 32) KERNEL<32>__VA_ARGS__;                        \
        else KERNEL<64>__VA_ARGS__;                                        \
    } while (0)

template <typename T>
GmresT<T>::GmresT(int64_t n, int m, Arena& ar, hipStream_t s) : n_(n), m_(m), ar_(&ar) {
    if (m < 1 || m > 63) throw Error(SCR_E_INVALID, "restart length must be in [1, 63]");
    V_ = ar.make<T>((size_t)(m + 1) * n);
    Z_ = ar.make<T>((size_t)m * n);
    GLay L{m};
    st_ = ar.make<double>(L.size());
    red_.init(n, ar, s);
    slot_.h = ar.ctx()->pinned.get();
    slot_.d = PinnedPool::device_ptr(slot_.h);
    slot_.h[15] = 0.0;
}
template <typename T>
GmresT<T>::~GmresT() {
    if (slot_.h) ar_->ctx()->pinned.put(slot_.h);
    ar_->free(V_); ar_->free(Z_); ar_->free(st_);
    red_.release(*ar_);
}

template <typename T>
KStat GmresT<T>::solve(OpT<T>& A, OpT<T>& M, const T* b, T* x, double tol, int maxit, bool use_x0, bool check_true,
                       hipStream_t s) {
    KStat st;
    const int64_t n = n_;
    const int m = m_;
    const int G = red_.grid;
    double* part = red_.partials;
    GLay L{m};
    double bn = device_norm(b, n, red_, slot_, s);
    if (!use_x0 || bn == 0.0) zero_dev(x, n * sizeof(T), s);
    if (bn == 0.0) {
        st.converged = true;
        return st;
    }
    if (!std::isfinite(bn)) throw Error(SCR_E_BREAKDOWN, "non-finite right-hand side");
    bool first = true;
    double est = INFINITY;
    int64_t nblk = cdiv(n, 256);
    for (;;) {
        T* V0 = V_;
        if (first && !use_x0) {
            copy_dev(V0, b, n * sizeof(T), s);
        } else {
            A.apply(x, V0, s);
            axpby_t_k<T><<<nblk, 256, 0, s>>>(n, 1.0, b, -1.0, V0);
        }
        first = false;
        dot_part_k<T><<<G, RTPB, 0, s>>>(n, V0, V0, part);
        gm_init_fin_k<<<1, RTPB, 0, s>>>(part, G, st_, m, slot_.d, slot_.next());
        check_launch("gm_init");
        slot_.wait(s);
        const double* host_ = slot_.h;
        double beta = host_[S_BETA];
        if (host_[S_FLAG] != 0.0) throw Error(SCR_E_BREAKDOWN, "non-finite residual in GMRES");
        st.rel_res = beta / bn;
        if (beta <= tol * bn) { st.converged = true; break; }
        if (!check_true && est <= tol * bn) { st.converged = true; break; }
        if (st.iters >= maxit) break;
        scale_by_k<<<nblk, 256, 0, s>>>(n, V0, st_ + L.scal() + S_INV);
        int j = 0;
        while (j < m) {
            T* Vj = V_ + (int64_t)j * n;
            T* Zj = Z_ + (int64_t)j * n;
            T* w = V_ + (int64_t)(j + 1) * n;
            M.apply(Vj, Zj, s);
            A.apply(Zj, w, s);
            int jn = j + 1;
            // CGS2: h1 = V^T w; w -= V h1, h2 = V^T w; w -= V h2; ||w||
            JDISPATCH(jn, mdot_k, <<<G, RTPB, 0, s>>>(n, jn, V_, n, w, part));
            JDISPATCH(jn, sum_k, <<<1, RTPB, 0, s>>>(part, G, jn, st_ + L.h1()));
            JDISPATCH(jn, upd_dot_k, <<<G, RTPB, 0, s>>>(n, jn, V_, n, w, st_ + L.h1(), part));
            JDISPATCH(jn, sum_k, <<<1, RTPB, 0, s>>>(part, G, jn, st_ + L.h2()));
            JDISPATCH(jn, upd_norm_k, <<<G, RTPB, 0, s>>>(n, jn, V_, n, w, st_ + L.h2(), part));
            arnoldi_fin_k<<<1, RTPB, 0, s>>>(part, G, st_, m, j, slot_.d, slot_.next());
            check_launch("cgs2");
            scale_by_k<<<nblk, 256, 0, s>>>(n, w, st_ + L.scal() + S_INV);
            slot_.wait(s);
            ++st.iters;
            ++j;
            if (host_[S_FLAG] != 0.0) throw Error(SCR_E_BREAKDOWN, "non-finite value in the Arnoldi process");
            est = host_[S_EST];
            if (host_[S_HN] == 0.0) break;   // happy breakdown: the Krylov space is invariant
            if (est <= tol * bn || st.iters >= maxit) break;
        }
        ysolve_k<<<1, 64, 0, s>>>(st_, m, j);
        maxpy_k<<<nblk, RTPB, 0, s>>>(n, j, Z_, n, st_ + L.y(), x);
        check_launch("gmres update");
        st.rel_res = est / bn;
        if (!check_true && (est <= tol * bn || st.iters >= maxit)) {
            st.converged = est <= tol * bn;
            break;
        }
    }
    return st;
}

template class GmresT<double>;
template class GmresT<float>;

// ------------------------------------------------------------------ CG on three columns
// Per-column state (doubles): RZ[3] | ALPHA[3] | BETA[3] | PQ[3] | DONE[3] | RN2[3] | spare
enum { C3_RZ = 0, C3_ALPHA = 3, C3_BETA = 6, C3_PQ = 9, C3_DONE = 12, C3_RN2 = 15, C3_SIZE = 32 };

// the reduction grid of a vector length (as Reducer::init)
static int reduce_grid(int64_t n) {
    int64_t g = cdiv(n, 4 * RTPB);
    return (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

// partials of x_c . y_c per column (the element order of dot_part_k, per column)
__global__ void __launch_bounds__(RTPB) dot3_part_k(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                                    double* __restrict__ partials) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * RTPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTPB)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += x[3 * i + c] * y[3 * i + c];
    block_partials<3>(acc, 3, partials);
}
__global__ void __launch_bounds__(RTPB) sum3_pub_k(const double* __restrict__ partials, int nblk, double* __restrict__ out,
                                                   double* __restrict__ hslot, double seq) {
    final_sums<3>(partials, nblk, 3, out);
    if (threadIdx.x == 0) publish(hslot, out, 3, seq);
}
// ALPHA_c = RZ_c / PQ_c for the columns still running
__global__ void __launch_bounds__(RTPB) cg3_alpha_fin_k(const double* __restrict__ partials, int nblk, double* __restrict__ st) {
    final_sums<3>(partials, nblk, 3, st + C3_PQ);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) st[C3_ALPHA + c] = st[C3_DONE + c] != 0.0 ? 0.0 : st[C3_RZ + c] / st[C3_PQ + c];
}
// per running column: (rold = r;) x += alpha p; r -= alpha q; partials of r . r
__global__ void __launch_bounds__(RTPB) cg3_update_k(int64_t n, double* __restrict__ x, const double* __restrict__ p,
                                                     double* __restrict__ r, const double* __restrict__ q,
                                                     double* __restrict__ rold, const double* __restrict__ st,
                                                     double* __restrict__ partials) {
    double alpha[3];
    bool run[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { alpha[c] = st[C3_ALPHA + c]; run[c] = st[C3_DONE + c] == 0.0; }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * RTPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTPB)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!run[c]) continue;
            const int64_t o = 3 * i + c;
            double ri = r[o];
            if (rold) rold[o] = ri;
            x[o] += alpha[c] * p[o];
            ri -= alpha[c] * q[o];
            r[o] = ri;
            acc[c] += ri * ri;
        }
    block_partials<3>(acc, 3, partials);
}
// partials of r_c . z_c and (flexible) z_c . (r_c - rold_c)
__global__ void __launch_bounds__(RTPB) cg3_rz_k(int64_t n, const double* __restrict__ r, const double* __restrict__ z,
                                                 const double* __restrict__ rold, double* __restrict__ partials) {
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * RTPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTPB)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double zi = z[3 * i + c], ri = r[3 * i + c];
            acc[c] += ri * zi;
            if (rold) acc[3 + c] += zi * (ri - rold[3 * i + c]);
        }
    block_partials<6>(acc, 6, partials);
}
// BETA_c = (flex ? num_c : rz_new_c) / RZ_c; RZ_c = rz_new_c   (init: only RZ)
__global__ void __launch_bounds__(RTPB) cg3_beta_fin_k(const double* __restrict__ partials, int nblk, int flexible,
                                                       int init, double* __restrict__ st) {
    __shared__ double res[6];
    final_sums<6>(partials, nblk, 6, res);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            if (st[C3_DONE + c] != 0.0) continue;
            if (!init) st[C3_BETA + c] = (flexible ? res[3 + c] : res[c]) / st[C3_RZ + c];
            st[C3_RZ + c] = res[c];
        }
}
__global__ void cg3_p_k(int64_t n3, double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ st) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n3) return;
    const int c = (int)(o % 3);
    p[o] = st[C3_DONE + c] != 0.0 ? 0.0 : z[o] + st[C3_BETA + c] * p[o];
}
__global__ void cg3_set_done_k(double* __restrict__ st, double d0, double d1, double d2) {
    if (threadIdx.x == 0) { st[C3_DONE] = d0; st[C3_DONE + 1] = d1; st[C3_DONE + 2] = d2; }
}
__global__ void cg3_init_k(double* __restrict__ st) {
    for (int e = threadIdx.x; e < C3_SIZE; e += blockDim.x) st[e] = 0.0;
}

int64_t Pcg3::workspace_doubles(int64_t n) {
    return 15 * n + C3_SIZE + (int64_t)reduce_grid(n) * RMAXJ + RMAXJ;
}

Pcg3::Pcg3(int64_t n, double* ws, StatusSlot* slot) : n_(n), grid_(reduce_grid(n)), slot_(slot) {
    r_ = ws; z_ = r_ + 3 * n; p_ = z_ + 3 * n; q_ = p_ + 3 * n; rold_ = q_ + 3 * n;
    st_ = rold_ + 3 * n;
    part_ = st_ + C3_SIZE;
    out_ = part_ + (int64_t)grid_ * RMAXJ;
}

Pcg3::Result Pcg3::solve(Op& A, Op& M, const double* b, double* x, double tol, int maxit, bool flexible,
                         hipStream_t s) {
    Result res;
    const int64_t n = n_;
    const int G = grid_;
    const int64_t nblk3 = cdiv(3 * n, 256);
    cg3_init_k<<<1, 64, 0, s>>>(st_);
    zero_dev(x, 3 * n * sizeof(double), s);
    dot3_part_k<<<G, RTPB, 0, s>>>(n, b, b, part_);
    sum3_pub_k<<<1, RTPB, 0, s>>>(part_, G, out_, slot_->d, slot_->next());
    check_launch("cg3 norm");
    slot_->wait(s);
    double bn[3];
    bool done[3];
    for (int c = 0; c < 3; ++c) {
        bn[c] = std::sqrt(slot_->h[c]);
        if (!std::isfinite(bn[c])) throw Error(SCR_E_BREAKDOWN, "non-finite right-hand side");
        done[c] = bn[c] == 0.0;
        res.converged[c] = done[c];
    }
    if (done[0] && done[1] && done[2]) return res;
    cg3_set_done_k<<<1, 64, 0, s>>>(st_, done[0] ? 1.0 : 0.0, done[1] ? 1.0 : 0.0, done[2] ? 1.0 : 0.0);
    copy_d(3 * n, b, r_, s);
    M.apply(r_, z_, s);
    copy_d(3 * n, z_, p_, s);
    cg3_rz_k<<<G, RTPB, 0, s>>>(n, r_, z_, nullptr, part_);
    cg3_beta_fin_k<<<1, RTPB, 0, s>>>(part_, G, 0, 1, st_);
    double* rold = flexible ? rold_ : nullptr;
    for (;;) {
        A.apply(p_, q_, s);
        dot3_part_k<<<G, RTPB, 0, s>>>(n, p_, q_, part_);
        cg3_alpha_fin_k<<<1, RTPB, 0, s>>>(part_, G, st_);
        cg3_update_k<<<G, RTPB, 0, s>>>(n, x, p_, r_, q_, rold, st_, part_);
        sum3_pub_k<<<1, RTPB, 0, s>>>(part_, G, st_ + C3_RN2, slot_->d, slot_->next());
        check_launch("cg3");
        slot_->wait(s);
        bool changed = false;
        for (int c = 0; c < 3; ++c) {
            if (done[c]) continue;
            ++res.iters[c];
            const double rn = std::sqrt(slot_->h[c]);
            if (!std::isfinite(rn)) throw Error(SCR_E_BREAKDOWN, "non-finite residual in CG");
            res.rel[c] = rn / bn[c];
            if (rn <= tol * bn[c]) { res.converged[c] = true; done[c] = true; changed = true; }
            else if (res.iters[c] >= maxit) { done[c] = true; changed = true; }
        }
        if (done[0] && done[1] && done[2]) break;
        if (changed)
            cg3_set_done_k<<<1, 64, 0, s>>>(st_, done[0] ? 1.0 : 0.0, done[1] ? 1.0 : 0.0, done[2] ? 1.0 : 0.0);
        M.apply(r_, z_, s);
        cg3_rz_k<<<G, RTPB, 0, s>>>(n, r_, z_, rold, part_);
        cg3_beta_fin_k<<<1, RTPB, 0, s>>>(part_, G, flexible ? 1 : 0, 0, st_);
        cg3_p_k<<<nblk3, 256, 0, s>>>(3 * n, p_, z_, st_);
        check_launch("cg3");
    }
    return res;
}

}  // namespace scr
