// sparse.hip -- scan/fill primitives, sliced-ELL layout, and the memory-bound sparse kernels of
// the solve phase: block SpMV/residual, fused smoother steps, restriction, coarse dense solve.
// Every kernel here streams matrix values once per call (HBM-bound, no MFMA: sparse products
// are not dense contractions).
#include "kernels.h"

namespace scr {

// ============================================================== primitives
constexpr int SCAN_TPB = 256, SCAN_PER = 4, SCAN_TILE = SCAN_TPB * SCAN_PER;

__global__ void scan_tile_sums(const int32_t* __restrict__ in, int64_t n, int64_t* __restrict__ sums) {
    __shared__ int64_t red[SCAN_TPB / WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
    for (int k = 0; k < SCAN_PER; ++k) {
        int64_t i = base + k * SCAN_TPB + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = wave_sum(s);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < SCAN_TPB / WAVE; ++w) t += red[w];
        sums[blockIdx.x] = t;
    }
}

// single block: exclusive scan of the tile sums (sequential over chunks of 256)
__global__ void scan_sums(int64_t* __restrict__ sums, int64_t nt) {
    __shared__ int64_t buf[SCAN_TPB];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nt; c0 += SCAN_TPB) {
        int64_t i = c0 + threadIdx.x;
        int64_t v = i < nt ? sums[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < SCAN_TPB; o <<= 1) {
            int64_t t = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nt) sums[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == SCAN_TPB - 1) carry += buf[SCAN_TPB - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nt] = carry;
}

__global__ void scan_tiles(const int32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ sums,
                           int32_t* __restrict__ out) {
    __shared__ int64_t buf[SCAN_TILE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int k = 0; k < SCAN_PER; ++k) {
        int64_t i = base + k * SCAN_TPB + threadIdx.x;
        buf[k * SCAN_TPB + threadIdx.x] = i < n ? in[i] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = sums[blockIdx.x];
        for (int t = 0; t < SCAN_TILE; ++t) {
            int64_t v = buf[t];
            buf[t] = run;
            run += v;
        }
    }
    __syncthreads();
    for (int k = 0; k < SCAN_PER; ++k) {
        int64_t i = base + k * SCAN_TPB + threadIdx.x;
        if (i < n) out[i] = (int32_t)buf[k * SCAN_TPB + threadIdx.x];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (int32_t)sums[gridDim.x];
}

int64_t scan_i32(const int32_t* in, int32_t* out, int64_t n, Arena& ar, hipStream_t s) {
    int64_t nt = cdiv(n, SCAN_TILE);
    if (nt == 0) {
        HIPCHK(hipMemsetAsync(out, 0, sizeof(int32_t), s));
        return 0;
    }
    int64_t* sums = ar.make<int64_t>(nt + 1);
    scan_tile_sums<<<nt, SCAN_TPB, 0, s>>>(in, n, sums);
    scan_sums<<<1, SCAN_TPB, 0, s>>>(sums, nt);
    scan_tiles<<<nt, SCAN_TPB, 0, s>>>(in, n, sums, out);
    check_launch("scan");
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, sums + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(sums);
    if (total > INT32_MAX) throw Error(SCR_E_INVALID, "index range exceeds int32");
    return total;
}

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
template <typename T>
void fill(T* p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    fill_kernel<T><<<cdiv(n, 256), 256, 0, s>>>(p, v, n);
    check_launch("fill");
}
template void fill<double>(double*, double, int64_t, hipStream_t);
template void fill<float>(float*, float, int64_t, hipStream_t);
template void fill<int64_t>(int64_t*, int64_t, int64_t, hipStream_t);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) { fill<int32_t>(p, v, n, s); }
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) { fill<uint8_t>(p, v, n, s); }

__global__ void cast_d2f_k(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void cast_f2d_k(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}
void cast_d2f(const double* a, float* b, int64_t n, hipStream_t s) {
    if (n > 0) cast_d2f_k<<<cdiv(n, 256), 256, 0, s>>>(a, b, n);
}
void cast_f2d(const float* a, double* b, int64_t n, hipStream_t s) {
    if (n > 0) cast_f2d_k<<<cdiv(n, 256), 256, 0, s>>>(a, b, n);
}

// ============================================================== sliced ELL
__global__ void sell_slice_len(const int32_t* __restrict__ rp, int64_t nr, int64_t nslices, int32_t* __restrict__ len) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices) return;
    int32_t m = 0;
    for (int64_t r = s * WAVE; r < (s + 1) * WAVE && r < nr; ++r) {
        int32_t l = rp[r + 1] - rp[r];
        m = l > m ? l : m;
    }
    len[s] = m;
}

template <typename T>
__global__ void sell_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ v,
                          int64_t nr, int64_t nc, int bb, const int32_t* __restrict__ off, int32_t* __restrict__ sci,
                          T* __restrict__ sv, int64_t nslices) {
    int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = row / WAVE;
    if (s >= nslices) return;
    int lane = (int)(row % WAVE);
    int64_t o0 = off[s], o1 = off[s + 1];
    int32_t lo = 0, hi = 0, pad = 0;
    if (row < nr) {
        lo = rp[row]; hi = rp[row + 1];
        pad = hi > lo ? ci[hi - 1] : (row < nc ? (int32_t)row : 0);
    }
    for (int64_t t = o0; t < o1; ++t) {
        int64_t q = lo + (t - o0);
        bool real = q < hi;
        sci[t * WAVE + lane] = real ? ci[q] : pad;
        for (int e = 0; e < bb; ++e) sv[(t * bb + e) * WAVE + lane] = real ? (T)v[q * bb + e] : (T)0;
    }
}

template <typename T>
DSell<T> sell_from_bsr(const DBsr& A, Arena& ar, hipStream_t s) {
    DSell<T> S;
    S.nr = A.nr; S.nc = A.nc; S.br = A.br; S.bc = A.bc; S.nnzb = A.nnzb;
    S.nslices = cdiv(A.nr, WAVE);
    if (S.nslices == 0) return S;
    int32_t* len = ar.make<int32_t>(S.nslices);
    sell_slice_len<<<cdiv(S.nslices, 256), 256, 0, s>>>(A.rp, A.nr, S.nslices, len);
    check_launch("sell_slice_len");
    S.off = ar.make<int32_t>(S.nslices + 1);
    S.slots = scan_i32(len, S.off, S.nslices, ar, s);
    ar.free(len);
    int bb = A.br * A.bc;
    S.ci = ar.make<int32_t>(S.slots * WAVE);
    S.v = ar.make<T>(S.slots * WAVE * bb);
    sell_fill<T><<<cdiv(S.nslices * WAVE, 256), 256, 0, s>>>(A.rp, A.ci, A.v, A.nr, A.nc, bb, S.off, S.ci, S.v,
                                                            S.nslices);
    check_launch("sell_fill");
    return S;
}
template <typename T>
void sell_free(DSell<T>& A, Arena& ar) {
    ar.free(A.off); ar.free(A.ci); ar.free(A.v);
    A = DSell<T>();
}
template DSell<double> sell_from_bsr<double>(const DBsr&, Arena&, hipStream_t);
template DSell<float> sell_from_bsr<float>(const DBsr&, Arena&, hipStream_t);
template void sell_free<double>(DSell<double>&, Arena&);
template void sell_free<float>(DSell<float>&, Arena&);

template <typename T>
__global__ void cast_vals(const double* __restrict__ a, T* __restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}
template <typename T>
DBsrT<T> bsrt_from_bsr(const DBsr& A, Arena& ar, hipStream_t s) {
    DBsrT<T> R;
    R.nr = A.nr; R.nc = A.nc; R.br = A.br; R.bc = A.bc; R.nnzb = A.nnzb;
    R.rp = A.rp; R.ci = A.ci;   // shares the index arrays of the FP64 matrix
    int64_t nv = A.nnzb * A.br * A.bc;
    R.v = ar.make<T>(nv);
    if (nv > 0) cast_vals<T><<<cdiv(nv, 256), 256, 0, s>>>(A.v, R.v, nv);
    check_launch("bsrt_from_bsr");
    return R;
}
template DBsrT<double> bsrt_from_bsr<double>(const DBsr&, Arena&, hipStream_t);
template DBsrT<float> bsrt_from_bsr<float>(const DBsr&, Arena&, hipStream_t);

// ============================================================== SpMV family (one lane per block row)
template <typename T, int BR, int BC, int MODE>
__global__ void __launch_bounds__(256) sell_mv_k(int64_t nr, int64_t nslices, const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                 const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y) {
    int64_t row = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    int64_t sl = row / WAVE;
    if (sl >= nslices) return;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t o0 = off[sl], o1 = off[sl + 1];
    T acc[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] = 0;
    for (int64_t t = o0; t < o1; ++t) {
        int64_t c = ci[t * WAVE + lane];
        T xv[BC];
#pragma unroll
        for (int k = 0; k < BC; ++k) xv[k] = x[c * BC + k];
        const T* vb = v + t * (BR * BC) * WAVE + lane;
#pragma unroll
        for (int r = 0; r < BR; ++r)
#pragma unroll
            for (int k = 0; k < BC; ++k) acc[r] += vb[(r * BC + k) * WAVE] * xv[k];
    }
    if (row >= nr) return;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        int64_t o = row * BR + r;
        if (MODE == 0) y[o] = acc[r];
        else if (MODE == 1) y[o] = b[o] - acc[r];
        else if (MODE == 2) y[o] += acc[r];
        else y[o] -= acc[r];
    }
}

template <typename T, int BR, int BC>
static void sell_mv_dispatch_mode(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s) {
    int64_t nblk = cdiv(A.nslices * WAVE, 256);
    if (nblk == 0) return;
    switch (mode) {
        case 0: sell_mv_k<T, BR, BC, 0><<<nblk, 256, 0, s>>>(A.nr, A.nslices, A.off, A.ci, A.v, x, b, y); break;
        case 1: sell_mv_k<T, BR, BC, 1><<<nblk, 256, 0, s>>>(A.nr, A.nslices, A.off, A.ci, A.v, x, b, y); break;
        case 2: sell_mv_k<T, BR, BC, 2><<<nblk, 256, 0, s>>>(A.nr, A.nslices, A.off, A.ci, A.v, x, b, y); break;
        default: sell_mv_k<T, BR, BC, 3><<<nblk, 256, 0, s>>>(A.nr, A.nslices, A.off, A.ci, A.v, x, b, y); break;
    }
    check_launch("sell_mv");
}

template <typename T>
void sell_mv(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s) {
    int key = A.br * 10 + A.bc;
    switch (key) {
        case 11: sell_mv_dispatch_mode<T, 1, 1>(A, x, b, y, mode, s); break;
        case 33: sell_mv_dispatch_mode<T, 3, 3>(A, x, b, y, mode, s); break;
        case 66: sell_mv_dispatch_mode<T, 6, 6>(A, x, b, y, mode, s); break;
        case 31: sell_mv_dispatch_mode<T, 3, 1>(A, x, b, y, mode, s); break;
        case 13: sell_mv_dispatch_mode<T, 1, 3>(A, x, b, y, mode, s); break;
        case 36: sell_mv_dispatch_mode<T, 3, 6>(A, x, b, y, mode, s); break;
        case 44: sell_mv_dispatch_mode<T, 4, 4>(A, x, b, y, mode, s); break;
        default: throw Error(SCR_E_UNIMPLEMENTED, "sell_mv: block shape " + std::to_string(A.br) + "x" + std::to_string(A.bc));
    }
}
template void sell_mv<double>(const DSell<double>&, const double*, const double*, double*, int, hipStream_t);
template void sell_mv<float>(const DSell<float>&, const float*, const float*, float*, int, hipStream_t);

// 4x4 system matrix on split vectors: x_v[3c..3c+2], x_p[c]
template <int MODE>
__global__ void __launch_bounds__(256) sell_mv_split4_k(int64_t nr, int64_t nslices, const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                        const double* __restrict__ x, const double* __restrict__ b,
                                                        double* __restrict__ y) {
    int64_t row = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    int64_t sl = row / WAVE;
    if (sl >= nslices) return;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t o0 = off[sl], o1 = off[sl + 1];
    const double* xp = x + 3 * nr;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = o0; t < o1; ++t) {
        int64_t c = ci[t * WAVE + lane];
        double xv[4] = {x[3 * c], x[3 * c + 1], x[3 * c + 2], xp[c]};
        const double* vb = v + t * 16 * WAVE + lane;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[r] += vb[(r * 4 + k) * WAVE] * xv[k];
    }
    if (row >= nr) return;
    int64_t o[4] = {3 * row, 3 * row + 1, 3 * row + 2, 3 * nr + row};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (MODE == 0) y[o[r]] = acc[r];
        else y[o[r]] = b[o[r]] - acc[r];
    }
}
void sell_mv_split4(const DSell<double>& K, const double* x, const double* b, double* y, int mode, hipStream_t s) {
    int64_t nblk = cdiv(K.nslices * WAVE, 256);
    if (nblk == 0) return;
    if (mode == 0) sell_mv_split4_k<0><<<nblk, 256, 0, s>>>(K.nr, K.nslices, K.off, K.ci, K.v, x, b, y);
    else sell_mv_split4_k<1><<<nblk, 256, 0, s>>>(K.nr, K.nslices, K.off, K.ci, K.v, x, b, y);
    check_launch("sell_mv_split4");
}

// ---------------------------------------------------------------- restriction (row per wave)
template <typename T, int BR, int BC>
__global__ void __launch_bounds__(256) bsrt_mv_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const T* __restrict__ v, const T* __restrict__ x, T* __restrict__ y) {
    int64_t row = xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x / WAVE);
    if (row >= nr) return;
    int lane = threadIdx.x & (WAVE - 1);
    T acc[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] = 0;
    for (int64_t q = rp[row] + lane; q < rp[row + 1]; q += WAVE) {
        int64_t c = ci[q];
        const T* vb = v + q * (BR * BC);
#pragma unroll
        for (int r = 0; r < BR; ++r)
#pragma unroll
            for (int k = 0; k < BC; ++k) acc[r] += vb[r * BC + k] * x[c * BC + k];
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
        T sum = wave_sum(acc[r]);
        if (lane == 0) y[row * BR + r] = sum;
    }
}
template <typename T>
void bsrt_mv(const DBsrT<T>& R, const T* x, T* y, hipStream_t s) {
    int64_t nblk = cdiv(R.nr, 4);
    if (nblk == 0) return;
    int key = R.br * 10 + R.bc;
    switch (key) {
        case 11: bsrt_mv_k<T, 1, 1><<<nblk, 256, 0, s>>>(R.nr, R.rp, R.ci, R.v, x, y); break;
        case 63: bsrt_mv_k<T, 6, 3><<<nblk, 256, 0, s>>>(R.nr, R.rp, R.ci, R.v, x, y); break;
        case 66: bsrt_mv_k<T, 6, 6><<<nblk, 256, 0, s>>>(R.nr, R.rp, R.ci, R.v, x, y); break;
        default: throw Error(SCR_E_UNIMPLEMENTED, "bsrt_mv: block shape");
    }
    check_launch("bsrt_mv");
}
template void bsrt_mv<double>(const DBsrT<double>&, const double*, double*, hipStream_t);
template void bsrt_mv<float>(const DBsrT<float>&, const float*, float*, hipStream_t);

// ---------------------------------------------------------------- fused smoother step
// dn = c1*d + c2*Dinv*(b - A xin) ; xout = xin + dn.  One lane per block row.
template <typename T, int B, bool RD, bool WD, bool ZERO>
__global__ void __launch_bounds__(256) smooth_k(int64_t nr, int64_t nslices, const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                const T* __restrict__ Dinv, const T* __restrict__ b,
                                                const T* __restrict__ xin, T* __restrict__ d, T* __restrict__ xout,
                                                T c1, T c2) {
    int64_t row = xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    int64_t sl = row / WAVE;
    if (sl >= nslices) return;
    int lane = threadIdx.x & (WAVE - 1);
    T r[B];
#pragma unroll
    for (int i = 0; i < B; ++i) r[i] = 0;
    if (!ZERO) {
        int64_t o0 = off[sl], o1 = off[sl + 1];
        for (int64_t t = o0; t < o1; ++t) {
            int64_t c = ci[t * WAVE + lane];
            T xv[B];
#pragma unroll
            for (int k = 0; k < B; ++k) xv[k] = xin[c * B + k];
            const T* vb = v + t * (B * B) * WAVE + lane;
#pragma unroll
            for (int i = 0; i < B; ++i)
#pragma unroll
                for (int k = 0; k < B; ++k) r[i] += vb[(i * B + k) * WAVE] * xv[k];
        }
    }
    if (row >= nr) return;
#pragma unroll
    for (int i = 0; i < B; ++i) r[i] = b[row * B + i] - r[i];
    const T* D = Dinv + row * (B * B);
#pragma unroll
    for (int i = 0; i < B; ++i) {
        T z = 0;
#pragma unroll
        for (int k = 0; k < B; ++k) z += D[i * B + k] * r[k];
        T dn = c2 * z;
        if (RD) dn += c1 * d[row * B + i];
        if (WD) d[row * B + i] = dn;
        xout[row * B + i] = ZERO ? dn : xin[row * B + i] + dn;
    }
}

template <typename T, int B>
static void smooth_dispatch(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, T c1, T c2,
                            bool rd, bool wd, bool zero, hipStream_t s) {
    int64_t nblk = cdiv(A.nslices * WAVE, 256);
    if (nblk == 0) return;
#define SK(RD, WD, Z) smooth_k<T, B, RD, WD, Z><<<nblk, 256, 0, s>>>(A.nr, A.nslices, A.off, A.ci, A.v, Dinv, b, xin, d, xout, c1, c2)
    if (zero) {
        if (wd) SK(false, true, true); else SK(false, false, true);
    } else if (rd) {
        if (wd) SK(true, true, false); else SK(true, false, false);
    } else {
        if (wd) SK(false, true, false); else SK(false, false, false);
    }
#undef SK
    check_launch("smooth_step");
}

template <typename T>
void smooth_step(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, double c1, double c2,
                 bool read_d, bool write_d, bool zero_in, hipStream_t s) {
    switch (A.br) {
        case 1: smooth_dispatch<T, 1>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s); break;
        case 3: smooth_dispatch<T, 3>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s); break;
        case 6: smooth_dispatch<T, 6>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s); break;
        default: throw Error(SCR_E_UNIMPLEMENTED, "smooth_step: block size");
    }
}
template void smooth_step<double>(const DSell<double>&, const double*, const double*, const double*, double*, double*,
                                  double, double, bool, bool, bool, hipStream_t);
template void smooth_step<float>(const DSell<float>&, const float*, const float*, const float*, float*, float*,
                                 double, double, bool, bool, bool, hipStream_t);

// ---------------------------------------------------------------- coarsest level: x = M b (M = A_c^-1, FP64)
template <typename T>
__global__ void __launch_bounds__(256) dense_mv_k(int64_t n, const double* __restrict__ M, const T* __restrict__ b,
                                                  T* __restrict__ x) {
    int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (row >= n) return;
    int lane = threadIdx.x & (WAVE - 1);
    double acc = 0.0;
    for (int64_t c = lane; c < n; c += WAVE) acc += M[row * n + c] * (double)b[c];
    acc = wave_sum(acc);
    if (lane == 0) x[row] = (T)acc;
}
template <typename T>
void dense_mv(int64_t n, const double* M, const T* b, T* x, hipStream_t s) {
    if (n <= 0) return;
    dense_mv_k<T><<<cdiv(n, 4), 256, 0, s>>>(n, M, b, x);
    check_launch("dense_mv");
}
template void dense_mv<double>(int64_t, const double*, const double*, double*, hipStream_t);
template void dense_mv<float>(int64_t, const double*, const float*, float*, hipStream_t);

// ---------------------------------------------------------------- input validation
// bits: 1 row_ptr, 2 column out of range, 4 unsorted/duplicate, 8 missing diagonal,
//       16 non-finite value, 32 zero on the velocity diagonal (bs 4) or the diagonal (bs 1)
__global__ void validate_k(int64_t nr, int bs, int64_t nnzb, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ v, int* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    int f = 0;
    int64_t lo = rp[i], hi = rp[i + 1];
    if (i == 0 && lo != 0) f |= 1;
    if (i == nr - 1 && hi != nnzb) f |= 1;
    if (lo < 0 || hi > nnzb || lo > hi) {
        atomicOr(flags, f | 1);
        return;
    }
    bool diag = false;
    int64_t prev = -1;
    int bb = bs * bs;
    for (int64_t q = lo; q < hi; ++q) {
        int64_t c = ci[q];
        if (c < 0 || c >= nr) { f |= 2; continue; }
        if (c <= prev) f |= 4;
        prev = c;
        for (int e = 0; e < bb; ++e)
            if (!isfinite(v[q * bb + e])) f |= 16;
        if (c == i) {
            diag = true;
            int nd = bs == 4 ? 3 : bs;   // the velocity diagonal (diag(A)) must be nonzero
            for (int k = 0; k < nd; ++k)
                if (v[q * bb + k * bs + k] == 0.0) f |= 32;
        }
    }
    if (!diag) f |= 8;
    if (f) atomicOr(flags, f);
}

int validate_bsr(int64_t nr, int bs, int64_t nnzb, const int32_t* rp, const int32_t* ci, const double* v, Arena& ar,
                 hipStream_t s) {
    int* flags = ar.make<int>(1);
    HIPCHK(hipMemsetAsync(flags, 0, sizeof(int), s));
    if (nr > 0) validate_k<<<cdiv(nr, 256), 256, 0, s>>>(nr, bs, nnzb, rp, ci, v, flags);
    check_launch("validate");
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(flags);
    return h;
}

}  // namespace scr
