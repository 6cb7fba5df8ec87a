// sparse.hip -- scan/fill primitives, sliced-ELL layout, and the memory-bound sparse kernels of
// the solve phase: block SpMV/residual, fused smoother steps, restriction, coarse dense solve.
// Every kernel here streams matrix values once per call (HBM-bound, no MFMA: sparse products
// are not dense contractions).
#include <hip/hip_ext.h>

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
        zero_dev(out, sizeof(int32_t), s);
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

// Device copies and zero fills by kernels (8-byte words when both ends and the size allow it,
// else bytes): the runtime's blit copy and fill leave a long idle gap behind them on the stream.
template <typename W>
__global__ void copy_words_k(int64_t n, const W* __restrict__ x, W* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}
template <typename W>
__global__ void zero_words_k(int64_t n, W* __restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
static unsigned word_grid(int64_t n) { return (unsigned)std::min<int64_t>(cdiv(n, 256), 16384); }
void copy_dev(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    if ((((uintptr_t)dst | (uintptr_t)src | bytes) & 7) == 0) {
        int64_t n = (int64_t)(bytes / 8);
        copy_words_k<uint64_t><<<word_grid(n), 256, 0, s>>>(n, (const uint64_t*)src, (uint64_t*)dst);
    } else {
        copy_words_k<uint8_t><<<word_grid((int64_t)bytes), 256, 0, s>>>((int64_t)bytes, (const uint8_t*)src, (uint8_t*)dst);
    }
    check_launch("copy_dev");
}
void zero_dev(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    if ((((uintptr_t)p | bytes) & 7) == 0) {
        int64_t n = (int64_t)(bytes / 8);
        zero_words_k<uint64_t><<<word_grid(n), 256, 0, s>>>(n, (uint64_t*)p);
    } else {
        zero_words_k<uint8_t><<<word_grid((int64_t)bytes), 256, 0, s>>>((int64_t)bytes, (uint8_t*)p);
    }
    check_launch("zero_dev");
}
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
// rank of block row i within its window: rows ordered by decreasing length, ties by index
__global__ void sell_rank_k(const int32_t* __restrict__ rp, int64_t nr, int64_t win, int32_t* __restrict__ rowid) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    int64_t w0 = (i / win) * win, w1 = w0 + win < nr ? w0 + win : nr;
    int32_t li = rp[i + 1] - rp[i];
    int64_t rank = 0;
    for (int64_t j = w0; j < w1; ++j) {
        int32_t lj = rp[j + 1] - rp[j];
        rank += (lj > li) || (lj == li && j < i);
    }
    rowid[w0 + rank] = (int32_t)i;
}

__global__ void sell_slice_len(const int32_t* __restrict__ rp, const int32_t* __restrict__ rowid, int rps,
                               int64_t nslices, int grp, int32_t* __restrict__ len) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices) return;
    int32_t m = 0;
    for (int64_t j = s * rps; j < (s + 1) * rps; ++j) {
        int32_t i = rowid[j];
        if (i < 0) continue;
        int32_t l = rp[i + 1] - rp[i];
        m = l > m ? l : m;
    }
    len[s] = (m + grp - 1) / grp * grp;
}

// Value k of slot t for lane `lane` in the scalar-row layout: k-major 64-wide vectors, except for
// 6-wide block rows.  FP64: the values in pairs (k, k+1) per lane, so that a lane reads two of
// them with one 16-byte load (measured: 6x6 FP64 smoother 33.6 -> 30.6 us per launch).  FP32: the
// first four values of a lane side by side (one 16-byte load), then the last two (one 8-byte load);
// pairs alone (three 8-byte loads) had been slower than six 4-byte loads, 17.5 -> 18.6 us.
__host__ __device__ __forceinline__ bool sell_paired(int bc, int elem_bytes) { return bc == 6; }
__host__ __device__ __forceinline__ int64_t sell_vidx(int64_t t, int k, int lane, int bc, bool paired, int elem_bytes) {
    if (paired && elem_bytes == 8) return ((t * 3 + (k >> 1)) * WAVE + lane) * 2 + (k & 1);
    if (paired) return t * 6 * WAVE + (k < 4 ? lane * 4 + k : 4 * WAVE + lane * 2 + (k - 4));
    return (t * bc + k) * WAVE + lane;
}

// 1x1 rows (one lane per row): slots grouped by four per lane, the column indices and the values of
// slots 4g .. 4g+3 of a lane side by side, so that a lane reads four indices with one 16-byte load
// and four values with one (FP32) or two (FP64); every slice holds a multiple of four slots.
constexpr int SELL_G = 4;
__host__ __device__ __forceinline__ int64_t sell_gpos(int64_t t, int lane) {
    return ((t >> 2) * WAVE + lane) * SELL_G + (t & 3);
}

// The fill kernels split a slice's slots into SELL_FILL_PARTS consecutive parts (multiples of four
// slots), one thread per (slice, part, lane): thread g of the grid takes slots [o0, o1) of the slice
// [ob, e1) that starts at o0 = ob on entry.
constexpr int SELL_FILL_PARTS = 4;
__device__ __forceinline__ void sell_fill_part(int64_t g, int64_t& o0, int64_t e1, int64_t& o1) {
    const int part = (int)((g / WAVE) % SELL_FILL_PARTS);
    const int64_t cs = ((e1 - o0 + SELL_FILL_PARTS - 1) / SELL_FILL_PARTS + SELL_G - 1) / SELL_G * SELL_G;
    o0 += part * cs;
    o1 = o0 + cs < e1 ? o0 + cs : e1;
}

template <typename T>
__global__ void sell_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ v,
                          int br, int bc, int rps, const int32_t* __restrict__ rowid, const int32_t* __restrict__ off,
                          int32_t* __restrict__ sci, T* __restrict__ sv, int64_t nslices) {
    const bool grouped = br == 1 && bc == 1;
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = g / (SELL_FILL_PARTS * WAVE);
    if (s >= nslices) return;
    int lane = (int)(g % WAVE);
    int j = lane / br;
    int r = lane % br;
    int64_t i = j < rps ? rowid[s * rps + j] : -1;
    bool valid = i >= 0;
    int64_t o0 = off[s], o1, e1 = off[s + 1];
    sell_fill_part(g, o0, e1, o1);
    if (o0 >= o1) return;
    int32_t lo = 0, hi = 0, pad = 0;
    if (valid) {
        lo = rp[i]; hi = rp[i + 1];
        pad = hi > lo ? ci[hi - 1] : 0;
    }
    const int64_t ob = off[s];   // first slot of the slice: slot t holds entry lo + (t - ob) of the row
    if (grouped) {
        // whole groups of four slots (the slice's slot range and each part are multiples of four)
        typedef int32_t I4 __attribute__((ext_vector_type(4)));
        typedef T V4 __attribute__((ext_vector_type(4)));
        for (int64_t t = o0; t < o1; t += SELL_G) {
            I4 cc;
            V4 vv;
#pragma unroll
            for (int u = 0; u < SELL_G; ++u) {
                const int64_t q = lo + (t + u - ob);
                const bool real = valid && q < hi;
                cc[u] = real ? ci[q] : pad;
                vv[u] = real ? (T)v[q] : (T)0;
            }
            *reinterpret_cast<I4*>(sci + sell_gpos(t, lane)) = cc;
            *reinterpret_cast<V4*>(sv + sell_gpos(t, lane)) = vv;
        }
        return;
    }
    bool colwriter = j < rps && r == 0;
    const bool paired = sell_paired(bc, (int)sizeof(T));
    for (int64_t t = o0; t < o1; ++t) {
        int64_t q = lo + (t - ob);
        bool real = valid && q < hi;
        if (colwriter) sci[t * rps + j] = real ? ci[q] : pad;
        for (int k = 0; k < bc; ++k)
            sv[sell_vidx(t, k, lane, bc, paired, (int)sizeof(T))] = real ? (T)v[(q * br + r) * bc + k] : (T)0;
    }
}

// Block-row lanes: the E = 3*bc values of slot t, in groups of g entries stored next to each
// other per lane (g = 2 for FP64, 4 for FP32), so that a lane reads a group with one 16-byte load
// (a wavefront 1 KB per load instruction); the last E % g entries as plain 64-wide vectors after
// the groups.
__host__ __device__ __forceinline__ int64_t rl_vidx(int64_t t, int e, int lane, int E, int g) {
    const int64_t base = t * E * WAVE;
    const int full = E - E % g;
    if (e < full) return base + (int64_t)(e / g) * g * WAVE + lane * g + (e % g);
    return base + (int64_t)e * WAVE + lane;
}

// block-row lanes: one thread per (slice, lane) = block row; all br*bc entries of each slot
template <typename T>
__global__ void sell_fill_rowlane(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const double* __restrict__ v, int nb2, const int32_t* __restrict__ rowid,
                                  const int32_t* __restrict__ off, int32_t* __restrict__ sci, T* __restrict__ sv,
                                  int64_t nslices) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = g / (SELL_FILL_PARTS * WAVE);
    if (s >= nslices) return;
    int lane = (int)(g % WAVE);
    const int64_t ob = off[s];
    int64_t o0 = ob, o1, e1 = off[s + 1];
    sell_fill_part(g, o0, e1, o1);
    if (o0 >= o1) return;
    int64_t i = rowid[s * WAVE + lane];
    int32_t lo = 0, hi = 0, pad = 0;
    if (i >= 0) {
        lo = rp[i]; hi = rp[i + 1];
        pad = hi > lo ? ci[hi - 1] : 0;
    }
    for (int64_t t = o0; t < o1; ++t) {
        int64_t q = lo + (t - ob);
        bool real = i >= 0 && q < hi;
        sci[t * WAVE + lane] = real ? ci[q] : pad;
        for (int e = 0; e < nb2; ++e)
            sv[rl_vidx(t, e, lane, nb2, sizeof(T) == 8 ? 2 : 4)] = real ? (T)v[q * nb2 + e] : (T)0;
    }
}

template <typename T>
DSell<T> sell_from_bsr(const DBsr& A, Arena& ar, hipStream_t s) {
    DSell<T> S;
    S.nr = A.nr; S.nc = A.nc; S.br = A.br; S.bc = A.bc; S.nnzb = A.nnzb;
    S.rowlane = A.br == 3 && (A.bc == 3 || A.bc == 6);
    S.rps = S.rowlane ? WAVE : WAVE / A.br;
    S.nslices = cdiv(A.nr, S.rps);
    if (S.nslices == 0) return S;
    S.rowid = ar.make<int32_t>(S.nslices * S.rps);
    fill_i32(S.rowid, -1, S.nslices * S.rps, s);
    int64_t win = (int64_t)(S.rowlane ? SELL_SIGMA_ROWLANE : SELL_SIGMA) * S.rps;
    sell_rank_k<<<cdiv(A.nr, 256), 256, 0, s>>>(A.rp, A.nr, win, S.rowid);
    int32_t* len = ar.make<int32_t>(S.nslices);
    const int grp = (!S.rowlane && A.br == 1 && A.bc == 1) ? SELL_G : 1;
    sell_slice_len<<<cdiv(S.nslices, 256), 256, 0, s>>>(A.rp, S.rowid, S.rps, S.nslices, grp, len);
    check_launch("sell_slice_len");
    S.off = ar.make<int32_t>(S.nslices + 1);
    S.slots = scan_i32(len, S.off, S.nslices, ar, s);
    ar.free(len);
    S.ci = ar.make<int32_t>(S.slots * S.rps + 1);
    if (S.rowlane) {
        S.v = ar.make<T>(S.slots * WAVE * A.br * A.bc + 1);
        sell_fill_rowlane<T><<<cdiv(S.nslices * SELL_FILL_PARTS * WAVE, 256), 256, 0, s>>>(A.rp, A.ci, A.v, A.br * A.bc, S.rowid, S.off,
                                                                        S.ci, S.v, S.nslices);
    } else {
        S.v = ar.make<T>(S.slots * WAVE * A.bc + 1);
        sell_fill<T><<<cdiv(S.nslices * SELL_FILL_PARTS * WAVE, 256), 256, 0, s>>>(A.rp, A.ci, A.v, A.br, A.bc, S.rps, S.rowid, S.off,
                                                                S.ci, S.v, S.nslices);
    }
    check_launch("sell_fill");
    return S;
}
template <typename T>
void sell_free(DSell<T>& A, Arena& ar) {
    ar.free(A.off); ar.free(A.rowid); ar.free(A.ci); ar.free(A.v);
    A = DSell<T>();
}
template DSell<double> sell_from_bsr<double>(const DBsr&, Arena&, hipStream_t);
template DSell<float> sell_from_bsr<float>(const DBsr&, Arena&, hipStream_t);
template void sell_free<double>(DSell<double>&, Arena&);
template void sell_free<float>(DSell<float>&, Arena&);

// row-entry-major values: entry e of the j-th block of row i at v[rp[i]*E + e*len_i + j]
// (E = br*bc), so that the lanes of a wave, one block each, read every entry coalesced
template <typename T>
__global__ void bsrt_fill_k(int64_t nr, int E, const int32_t* __restrict__ rp, const double* __restrict__ a,
                            T* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (i >= nr) return;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t q0 = rp[i], len = rp[i + 1] - q0;
    for (int64_t j = lane; j < len; j += WAVE)
        for (int e = 0; e < E; ++e) b[q0 * E + e * len + j] = (T)a[(q0 + j) * E + e];
}
template <typename T>
DBsrT<T> bsrt_from_bsr(const DBsr& A, Arena& ar, hipStream_t s) {
    DBsrT<T> R;
    R.nr = A.nr; R.nc = A.nc; R.br = A.br; R.bc = A.bc; R.nnzb = A.nnzb;
    R.rp = A.rp; R.ci = A.ci;   // shares the index arrays of the FP64 matrix
    int64_t nv = A.nnzb * A.br * A.bc;
    R.v = ar.make<T>(nv > 0 ? nv : 1);
    if (nv > 0) bsrt_fill_k<T><<<cdiv(A.nr, 4), 256, 0, s>>>(A.nr, A.br * A.bc, A.rp, A.v, R.v);
    check_launch("bsrt_from_bsr");
    return R;
}
template DBsrT<double> bsrt_from_bsr<double>(const DBsr&, Arena&, hipStream_t);
template DBsrT<float> bsrt_from_bsr<float>(const DBsr&, Arena&, hipStream_t);

// ============================================================== SpMV family (one lane per scalar row)
// Unrolled slot loop: U slots' columns, then their values and x segments, are loaded before use.
// Matrix values are read once per call: nontemporal loads keep them from evicting the gathered
// x entries and the per-row vectors from the caches.
// (measured: a gain for 3- and 6-wide FP64 row segments, a loss for scalar entries)
template <int BC, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    if (BC >= 3 && sizeof(T) == 8) return __builtin_nontemporal_load(p);
    return *p;
}
template <int BC> struct Unroll { static constexpr int U = BC == 1 ? 8 : (BC <= 4 ? 4 : 2); };

// the BC values of slot t of a lane (layout of sell_vidx)
template <typename T, int BC>
__device__ __forceinline__ void sell_vals(const T* __restrict__ v, int64_t t, int lane, T (&vv)[BC]) {
    if constexpr (BC == 6 && sizeof(T) == 8) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        const V2* vp = reinterpret_cast<const V2*>(v);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            const V2 w = __builtin_nontemporal_load(vp + (t * 3 + kk) * WAVE + lane);
            vv[2 * kk] = w.x;
            vv[2 * kk + 1] = w.y;
        }
    } else if constexpr (BC == 6) {
        typedef T V4 __attribute__((ext_vector_type(4)));
        typedef T V2 __attribute__((ext_vector_type(2)));
        const T* base = v + t * 6 * WAVE;
        const V4 a = __builtin_nontemporal_load(reinterpret_cast<const V4*>(base) + lane);
        const V2 c = __builtin_nontemporal_load(reinterpret_cast<const V2*>(base + 4 * WAVE) + lane);
        vv[0] = a.x; vv[1] = a.y; vv[2] = a.z; vv[3] = a.w;
        vv[4] = c.x; vv[5] = c.y;
    } else {
#pragma unroll
        for (int k = 0; k < BC; ++k) vv[k] = ld_stream<BC>(v + (t * BC + k) * WAVE + lane);
    }
}

// the four column indices and the four values of slot group g of a lane (layout of sell_gpos)
typedef int32_t SellI4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ SellI4 sell_gidx(const int32_t* __restrict__ ci, int64_t g, int lane) {
    return *reinterpret_cast<const SellI4*>(ci + (g * WAVE + lane) * SELL_G);
}
template <typename T>
__device__ __forceinline__ void sell_gvals(const T* __restrict__ v, int64_t g, int lane, T (&vv)[SELL_G]) {
    const T* p = v + (g * WAVE + lane) * SELL_G;
    if constexpr (sizeof(T) == 8) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        const V2 a = reinterpret_cast<const V2*>(p)[0], b = reinterpret_cast<const V2*>(p)[1];
        vv[0] = a.x; vv[1] = a.y; vv[2] = b.x; vv[3] = b.y;
    } else {
        typedef T V4 __attribute__((ext_vector_type(4)));
        const V4 a = *reinterpret_cast<const V4*>(p);
        vv[0] = a.x; vv[1] = a.y; vv[2] = a.z; vv[3] = a.w;
    }
}

// sell_row_dot for 1x1 rows in the grouped layout (o0, o1 multiples of four): two groups (eight
// slots) per step, the indices one step ahead; the terms are added in slot order, as in the
// one-slot-at-a-time loop
template <typename T, typename XF>
__device__ __forceinline__ T sell_row_dot_g(int64_t o0, int64_t o1, int lane, const int32_t* __restrict__ ci,
                                            const T* __restrict__ v, XF xat) {
    T acc = 0;
    const int64_t g1 = o1 / SELL_G;
    int64_t g = o0 / SELL_G;
    SellI4 c[2];
    if (g + 2 <= g1) {
        c[0] = sell_gidx(ci, g, lane);
        c[1] = sell_gidx(ci, g + 1, lane);
    }
    for (; g + 2 <= g1; g += 2) {
        T xx[2][SELL_G], vv[2][SELL_G];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < SELL_G; ++j) xx[u][j] = xat((int64_t)c[u][j], 0);
        SellI4 cn[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) cn[u] = sell_gidx(ci, g + 2 + u < g1 ? g + 2 + u : g1 - 1, lane);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) sell_gvals<T>(v, g + u, lane, vv[u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < SELL_G; ++j) acc += vv[u][j] * xx[u][j];
#pragma unroll
        for (int u = 0; u < 2; ++u) c[u] = cn[u];
    }
    for (; g < g1; ++g) {
        const SellI4 cc = sell_gidx(ci, g, lane);
        T vv[SELL_G];
        sell_gvals<T>(v, g, lane, vv);
#pragma unroll
        for (int j = 0; j < SELL_G; ++j) acc += vv[j] * xat((int64_t)cc[j], 0);
    }
    return acc;
}

// acc = sum over the lane's row segments of v . x[col*BC : col*BC+BC]; cl = the lane's block row
// within the slice (column indices are stored once per block row, RPS per slot)
template <typename T, int BC, int RPS, typename XF>
__device__ __forceinline__ T sell_row_dot(int64_t o0, int64_t o1, int lane, int cl, const int32_t* __restrict__ ci,
                                          const T* __restrict__ v, XF xat) {
    if constexpr (BC == 1 && RPS == WAVE) return sell_row_dot_g<T>(o0, o1, lane, ci, v, xat);
    constexpr int U = Unroll<BC>::U;
    T acc = 0;
    int64_t t = o0;
    // software-pipelined as the block-row-lane loop: column indices one step ahead, x gathers and
    // the next indices issued before the values, one memory round trip per step
    int32_t c[U];     // int32 until used, so that no sign extension waits for the load
    if (t + U <= o1) {
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = ci[(t + u) * RPS + cl];
    }
    for (; t + U <= o1; t += U) {
        T xx[U][BC], vv[U][BC];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < BC; ++k) xx[u][k] = xat((int64_t)c[u], k);
        int32_t cn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t q = t + U + u < o1 ? t + U + u : o1 - 1;     // stays inside the slice
            cn[u] = ci[q * RPS + cl];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) sell_vals<T, BC>(v, t + u, lane, vv[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < BC; ++k) acc += vv[u][k] * xx[u][k];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cn[u];
    }
    for (; t < o1; ++t) {
        int64_t c = ci[t * RPS + cl];
        T vv[BC];
        sell_vals<T, BC>(v, t, lane, vv);
#pragma unroll
        for (int k = 0; k < BC; ++k) acc += vv[k] * xat(c, k);
    }
    return acc;
}

// WPS waves share one slice when a matrix has too few slices to fill the chip (coarse levels):
// wave w of the group takes the w-th contiguous chunk of the slice's slots, and the partial row
// sums are added in LDS in the fixed order w = 0, 1, ... (deterministic).
// slices per workgroup and threads per workgroup for WPS waves per slice (at least 256 threads)
template <int WPS> struct SliceGroup {
    static constexpr int SPB = WPS >= 4 ? 1 : 4 / WPS;
    static constexpr int THREADS = SPB * WPS * 64;
};
// (G = SELL_G for the grouped 1x1 layout: the chunks start at whole slot groups)
template <int WPS, int G = 1>
__device__ __forceinline__ void slice_part(int64_t o0, int64_t o1, int part, int64_t& a, int64_t& b) {
    int64_t len = (o1 - o0) / G;
    a = o0 + G * (len * part / WPS);
    b = o0 + G * (len * (part + 1) / WPS);
}

template <typename T, int BR, int BC, int MODE, int WPS>
__global__ void __launch_bounds__(SliceGroup<WPS>::THREADS) sell_mv_k(int64_t nslices, const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ rowid, const int32_t* __restrict__ ci,
                                                 const T* __restrict__ v, const T* __restrict__ x,
                                                 const T* __restrict__ b, T* __restrict__ y) {
    constexpr int RPS = WAVE / BR;
    int wv = threadIdx.x / WAVE;
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * SliceGroup<WPS>::SPB + wv / WPS;
    int lane = threadIdx.x & (WAVE - 1);
    bool live = sl < nslices;
    auto xat = [&](int64_t c, int k) { return x[c * BC + k]; };
    int cl = lane / BR < RPS ? lane / BR : RPS - 1;
    T acc = 0;
    if (live) {
        int64_t a, e;
        slice_part<WPS, (BR == 1 && BC == 1) ? SELL_G : 1>(off[sl], off[sl + 1], wv % WPS, a, e);
        acc = sell_row_dot<T, BC, RPS>(a, e, lane, cl, ci, v, xat);
    }
    if (WPS > 1) {
        __shared__ T red[SliceGroup<WPS>::SPB * WPS][WAVE];
        red[wv][lane] = acc;
        __syncthreads();
        if (wv % WPS != 0) return;
        for (int w = 1; w < WPS; ++w) acc += red[wv + w][lane];
    }
    if (!live || lane >= RPS * BR) return;
    int64_t i = rowid[sl * RPS + cl];
    if (i < 0) return;
    int64_t o = i * BR + lane % BR;
    if (MODE == 0) y[o] = acc;
    else if (MODE == 1) y[o] = b[o] - acc;
    else if (MODE == 2) y[o] += acc;
    else y[o] -= acc;
}

// waves per slice: doubled while the matrix has fewer than 64K waves in all (256 per CU) and each
// wave keeps at least 3 of the slice's average slots, up to 8 waves per slice; on small matrices
// (fewer than 512 slices, where the time is the latency of each wave's chain of dependent loads)
// at least 4 slots and up to 16 waves.  Measured on the refined tube (A/B on one box): a cap of 64K
// instead of 16K waves puts 8 waves on each slice of AMG(A)'s level 1 (55 slots) and 4 on AMG(S^)'s
// level 0 and makes the FP64 solve 5 % faster; 16 waves per slice on level 1 is slower again.
template <typename T>
static int waves_per_slice(const DSell<T>& A) {
    if (A.nslices <= 0) return 1;
    int64_t avg = A.slots / A.nslices;
    int wmax = A.nslices < 512 ? 16 : 8, per = A.nslices < 512 ? 4 : 3;
    int w = 1;
    while (w < wmax && A.nslices * w < 65536 && avg >= per * (w * 2)) w *= 2;
    return w;
}

// ---- block-row lanes (3xBC, BC = 3 or 6): r[0..2] = sum over the lane's slots of block * x[col]
// Two slots per step (both slots' columns, then their values and x vectors are loaded before
// use); FP32 3x6 takes one slot per step (18 values and an x 6-vector).  Measured on the refined
// tube: two 3x6 FP64 slots per step make the level-0 prolongation 3.5 % faster.  FP64 values are
// streamed with nontemporal loads (read once per call; measured: a gain in FP64, a loss in FP32).
// CAP: also copy the 3x3 block of column irow (the diagonal block of the lane's row) into dg; the
// first match is the stored block (padding slots that repeat the row's last column hold zeros and
// come after it)
template <typename T, int BC, bool CAP = false>
__device__ __forceinline__ void rowlane3_dot(int64_t t, int64_t o1, int lane, const int32_t* __restrict__ ci,
                                             const T* __restrict__ v, const T* __restrict__ x, T r[3],
                                             int32_t irow = -1, T* dg = nullptr) {
    constexpr int U = (BC == 3 || sizeof(T) == 8) ? 2 : 1, E = 3 * BC;
    // the E values of slot tt (layout of rl_vidx): FP64 in 16-byte pairs, FP32 in 16-byte quads,
    // nontemporal
    auto load_slot = [&](int64_t tt, T (&vv)[E]) {
        if constexpr (sizeof(T) == 8) {
            typedef T V2 __attribute__((ext_vector_type(2)));
            const T* base = v + tt * E * WAVE;
#pragma unroll
            for (int k = 0; k < E / 2; ++k) {
                const V2 w = __builtin_nontemporal_load(reinterpret_cast<const V2*>(base + k * 2 * WAVE) + lane);
                vv[2 * k] = w.x;
                vv[2 * k + 1] = w.y;
            }
            if constexpr (E % 2 == 1) vv[E - 1] = __builtin_nontemporal_load(base + (E - 1) * WAVE + lane);
        } else {
            typedef T V4 __attribute__((ext_vector_type(4)));
            const T* base = v + tt * E * WAVE;
#pragma unroll
            for (int k = 0; k < E / 4; ++k) {
                const V4 w = __builtin_nontemporal_load(reinterpret_cast<const V4*>(base + k * 4 * WAVE) + lane);
                vv[4 * k] = w.x;
                vv[4 * k + 1] = w.y;
                vv[4 * k + 2] = w.z;
                vv[4 * k + 3] = w.w;
            }
#pragma unroll
            for (int e = E - E % 4; e < E; ++e) vv[e] = __builtin_nontemporal_load(base + e * WAVE + lane);
        }
    };
    auto fma_block = [&](const T* vv, const T* xx) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            T sum = vv[BC * q] * xx[0];
#pragma unroll
            for (int k = 1; k < BC; ++k) sum += vv[BC * q + k] * xx[k];
            r[q] += sum;
        }
    };
    r[0] = r[1] = r[2] = 0;
    bool got = false;
    (void)got;
    // software-pipelined: the column indices of a step are loaded one step ahead, so each step
    // issues its x gathers, the next step's indices and its values together and waits once
    int32_t c[U];     // int32 until used, so that no sign extension waits for the load
    if (t + U <= o1) {
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = ci[(t + u) * WAVE + lane];
    }
    for (; t + U <= o1; t += U) {
        T vv[U][E], xx[U][BC];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < BC; ++k) xx[u][k] = x[(int64_t)c[u] * BC + k];
        int32_t cn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t q = t + U + u < o1 ? t + U + u : o1 - 1;     // stays inside the slice
            cn[u] = ci[q * WAVE + lane];
        }
        __builtin_amdgcn_sched_barrier(0);     // keep the gathers and indices ahead of the values
#pragma unroll
        for (int u = 0; u < U; ++u) load_slot(t + u, vv[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) fma_block(vv[u], xx[u]);
        if constexpr (CAP) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c[u] == irow && !got) {
#pragma unroll
                    for (int e = 0; e < 9; ++e) dg[e] = vv[u][e];
                    got = true;
                }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cn[u];
    }
    if (U > 1 && t < o1) {
        int64_t c = ci[t * WAVE + lane];
        T vv[E], xx[BC];
        load_slot(t, vv);
#pragma unroll
        for (int k = 0; k < BC; ++k) xx[k] = x[c * BC + k];
        fma_block(vv, xx);
        if constexpr (CAP) {
            if (c == irow && !got) {
#pragma unroll
                for (int e = 0; e < 9; ++e) dg[e] = vv[e];
            }
        }
    }
}

template <typename T, int BC, int MODE>
__global__ void __launch_bounds__(256) sell_mv_rl3_k(int64_t nslices, const int32_t* __restrict__ off,
                                                     const int32_t* __restrict__ rowid, const int32_t* __restrict__ ci,
                                                     const T* __restrict__ v, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y) {
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * 4 + threadIdx.x / WAVE;
    if (sl >= nslices) return;
    int lane = threadIdx.x & (WAVE - 1);
    T r[3];
    rowlane3_dot<T, BC>(off[sl], off[sl + 1], lane, ci, v, x, r);
    int64_t i = rowid[sl * WAVE + lane];
    if (i < 0) return;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int64_t o = i * 3 + q;
        if (MODE == 0) y[o] = r[q];
        else if (MODE == 1) y[o] = b[o] - r[q];
        else if (MODE == 2) y[o] += r[q];
        else y[o] -= r[q];
    }
}

template <typename T, int BR, int BC>
static void sell_mv_dispatch_mode(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s) {
    // splitting slices only pays on the square coarse-level shapes (6x6 A levels, 1x1 S^/L levels)
    constexpr bool SPLIT = (BR == 6 && BC == 6) || (BR == 1 && BC == 1);
    int wps = SPLIT ? waves_per_slice(A) : 1;
    if (A.nslices == 0) return;
#define MV(W)                                                                                                  \
    {                                                                                                          \
        constexpr int W_ = W;                                                                                  \
        int64_t nblk = cdiv(A.nslices, SliceGroup<W_>::SPB);                                                   \
        dim3 g((unsigned)nblk), t(SliceGroup<W_>::THREADS);                                                     \
        switch (mode) {                                                                                        \
            case 0: sell_mv_k<T, BR, BC, 0, W_><<<g, t, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
            case 1: sell_mv_k<T, BR, BC, 1, W_><<<g, t, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
            case 2: sell_mv_k<T, BR, BC, 2, W_><<<g, t, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
            default: sell_mv_k<T, BR, BC, 3, W_><<<g, t, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
        }                                                                                                      \
    }
    if (!SPLIT || wps == 1) MV(1)
    else if (wps == 2) MV((SPLIT ? 2 : 1))
    else if (wps == 4) MV((SPLIT ? 4 : 1))
    else if (wps == 8) MV((SPLIT ? 8 : 1))
    else MV((SPLIT ? 16 : 1))
#undef MV
    check_launch("sell_mv");
}

template <typename T>
void sell_mv(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s) {
    if (A.rowlane) {
        int64_t nblk = cdiv(A.nslices, 4);
        if (nblk == 0) return;
#define RL(BC)                                                                                                     \
    switch (mode) {                                                                                                \
        case 0: sell_mv_rl3_k<T, BC, 0><<<nblk, 256, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
        case 1: sell_mv_rl3_k<T, BC, 1><<<nblk, 256, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
        case 2: sell_mv_rl3_k<T, BC, 2><<<nblk, 256, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
        default: sell_mv_rl3_k<T, BC, 3><<<nblk, 256, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
    }
        if (A.bc == 3) { RL(3) } else { RL(6) }
#undef RL
        check_launch("sell_mv");
        return;
    }
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

// 4x4 system matrix on split vectors [x_v (3n); x_p (n)]
template <int MODE>
__global__ void __launch_bounds__(256) sell_mv_split4_k(int64_t nr, int64_t nslices, const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ rowid,
                                                        const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                        const double* __restrict__ x, const double* __restrict__ b,
                                                        double* __restrict__ y) {
    constexpr int RPS = WAVE / 4;
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * 4 + threadIdx.x / WAVE;
    if (sl >= nslices) return;
    int lane = threadIdx.x & (WAVE - 1);
    const double* xp = x + 3 * nr;
    auto xat = [&](int64_t c, int k) { return k < 3 ? x[3 * c + k] : xp[c]; };
    double acc = sell_row_dot<double, 4, RPS>(off[sl], off[sl + 1], lane, lane / 4, ci, v, xat);
    int64_t i = rowid[sl * RPS + lane / 4];
    if (i < 0) return;
    int r = lane & 3;
    int64_t o = r < 3 ? 3 * i + r : 3 * nr + i;
    if (MODE == 0) y[o] = acc;
    else y[o] = b[o] - acc;
}
void sell_mv_split4(const DSell<double>& K, const double* x, const double* b, double* y, int mode, hipStream_t s) {
    int64_t nblk = cdiv(K.nslices, 4);
    if (nblk == 0) return;
    if (mode == 0) sell_mv_split4_k<0><<<nblk, 256, 0, s>>>(K.nr, K.nslices, K.off, K.rowid, K.ci, K.v, x, b, y);
    else sell_mv_split4_k<1><<<nblk, 256, 0, s>>>(K.nr, K.nslices, K.off, K.rowid, K.ci, K.v, x, b, y);
    check_launch("sell_mv_split4");
}

// ---------------------------------------------------------------- restriction (row per wave)
// Values in row-entry-major order (bsrt_fill_k); lane j of the wave takes blocks j, j+64, ...
template <typename T, int BR, int BC>
__global__ void __launch_bounds__(256) bsrt_mv_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const T* __restrict__ v, const T* __restrict__ x, T* __restrict__ y) {
    int64_t row = xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x / WAVE);
    if (row >= nr) return;
    int lane = threadIdx.x & (WAVE - 1);
    T acc[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) acc[r] = 0;
    int64_t q0 = rp[row], len = rp[row + 1] - q0;
    for (int64_t j = lane; j < len; j += WAVE) {
        int64_t c = ci[q0 + j];
        const T* vb = v + q0 * (BR * BC) + j;
        T xx[BC];
#pragma unroll
        for (int k = 0; k < BC; ++k) xx[k] = x[c * BC + k];
#pragma unroll
        for (int r = 0; r < BR; ++r)
#pragma unroll
            for (int k = 0; k < BC; ++k) acc[r] += ld_stream<BC>(vb + (r * BC + k) * len) * xx[k];
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
// dn = c1*d + c2*Dinv*(b - A xin) ; xout = xin + dn.  One lane per scalar row; the block
// residual of a block row is gathered from its B lanes with shuffles to apply Dinv.
template <typename T, int B, bool RD, bool WD, bool ZERO, int WPS>
__global__ void __launch_bounds__(SliceGroup<WPS>::THREADS) smooth_k(int64_t nslices, const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ rowid,
                                                const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                const T* __restrict__ Dinv, const T* __restrict__ b,
                                                const T* __restrict__ xin, T* __restrict__ d, T* __restrict__ xout,
                                                T c1, T c2) {
    constexpr int RPS = WAVE / B;
    int wv = threadIdx.x / WAVE;
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * SliceGroup<WPS>::SPB + wv / WPS;
    bool live = sl < nslices;
    int lane = threadIdx.x & (WAVE - 1);
    int cl = lane / B < RPS ? lane / B : RPS - 1;
    T acc = 0;
    if (!ZERO && live) {
        auto xat = [&](int64_t c, int k) { return xin[c * B + k]; };
        int64_t a, e;
        slice_part<WPS, B == 1 ? SELL_G : 1>(off[sl], off[sl + 1], wv % WPS, a, e);
        acc = sell_row_dot<T, B, RPS>(a, e, lane, cl, ci, v, xat);
    }
    if (WPS > 1) {
        __shared__ T red[SliceGroup<WPS>::SPB * WPS][WAVE];
        red[wv][lane] = acc;
        __syncthreads();
        if (wv % WPS != 0) return;
        for (int w = 1; w < WPS; ++w) acc += red[wv + w][lane];
    }
    if (!live) return;
    int64_t i = rowid[sl * RPS + cl];
    int r = lane % B;
    bool valid = lane < RPS * B && i >= 0;
    int64_t o = i * B + r;
    T res = valid ? b[o] - acc : (T)0;
    T z = 0;
    int base = lane - r;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        T rk = B == 1 ? res : __shfl(res, base + k, WAVE);
        if (valid) z += Dinv[o * B + k] * rk;
    }
    if (!valid) return;
    T dn = c2 * z;
    if (RD) dn += c1 * d[o];
    if (WD) d[o] = dn;
    xout[o] = ZERO ? dn : xin[o] + dn;
}

// block-row lanes (3x3): the lane holds its block row's whole residual, so D^-1 applies in-lane
template <typename T, bool RD, bool WD, bool ZERO>
__global__ void __launch_bounds__(256) smooth_rl3_k(int64_t nslices, const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ rowid,
                                                    const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                    const T* __restrict__ Dinv, const T* __restrict__ b,
                                                    const T* __restrict__ xin, T* __restrict__ d, T* __restrict__ xout,
                                                    T c1, T c2) {
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * 4 + threadIdx.x / WAVE;
    if (sl >= nslices) return;
    int lane = threadIdx.x & (WAVE - 1);
    T r[3] = {0, 0, 0};
    const int64_t i = rowid[sl * WAVE + lane];
    // the diagonal block is captured while the row streams by and D^-1 is not read (72 bytes per
    // row less; measured on the refined tube: the FP64 steps 6-11 % faster, FP32 mixed solves 1.6 %)
    constexpr bool CAP = true;
    T dg[9];
    if (!ZERO) rowlane3_dot<T, 3, CAP>(off[sl], off[sl + 1], lane, ci, v, xin, r, (int32_t)i, dg);
    if (i < 0) return;
    T res[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) res[q] = b[i * 3 + q] - r[q];
    // z = D^-1 res: the adjugate of the captured block over its determinant (the stored inverse in
    // the first step, which has no matrix product)
    T z[3];
    if (ZERO || !CAP) {
        const T* Di = Dinv + i * 9;
#pragma unroll
        for (int q = 0; q < 3; ++q) z[q] = Di[3 * q] * res[0] + Di[3 * q + 1] * res[1] + Di[3 * q + 2] * res[2];
    } else {
        const T a0 = dg[4] * dg[8] - dg[5] * dg[7], a1 = dg[2] * dg[7] - dg[1] * dg[8], a2 = dg[1] * dg[5] - dg[2] * dg[4];
        const T a3 = dg[5] * dg[6] - dg[3] * dg[8], a4 = dg[0] * dg[8] - dg[2] * dg[6], a5 = dg[2] * dg[3] - dg[0] * dg[5];
        const T a6 = dg[3] * dg[7] - dg[4] * dg[6], a7 = dg[1] * dg[6] - dg[0] * dg[7], a8 = dg[0] * dg[4] - dg[1] * dg[3];
        const T inv = T(1) / (dg[0] * a0 + dg[1] * a3 + dg[2] * a6);
        z[0] = (a0 * res[0] + a1 * res[1] + a2 * res[2]) * inv;
        z[1] = (a3 * res[0] + a4 * res[1] + a5 * res[2]) * inv;
        z[2] = (a6 * res[0] + a7 * res[1] + a8 * res[2]) * inv;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int64_t o = i * 3 + q;
        T dn = c2 * z[q];
        if (RD) dn += c1 * d[o];
        if (WD) d[o] = dn;
        xout[o] = ZERO ? dn : xin[o] + dn;
    }
}

template <typename T>
static void smooth_rl3(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, T c1, T c2,
                       bool rd, bool wd, bool zero, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    int64_t nblk = cdiv(A.nslices, 4);
    if (nblk == 0) return;
#define SK(RD, WD, Z)                                                                                              \
    do {                                                                                                           \
        if (e0)                                                                                                    \
            hipExtLaunchKernelGGL((smooth_rl3_k<T, RD, WD, Z>), dim3((unsigned)nblk), dim3(256), 0, s, e0, e1, 0,  \
                                  A.nslices, (const int32_t*)A.off, (const int32_t*)A.rowid, (const int32_t*)A.ci, \
                                  (const T*)A.v, Dinv, b, xin, d, xout, c1, c2);                                   \
        else                                                                                                       \
            smooth_rl3_k<T, RD, WD, Z><<<nblk, 256, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, Dinv, b, xin, d, \
                                                           xout, c1, c2);                                          \
    } while (0)
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

template <typename T, int B>
static void smooth_dispatch(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, T c1, T c2,
                            bool rd, bool wd, bool zero, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    int wps = zero ? 1 : waves_per_slice(A);
    if (A.nslices == 0) return;
#define SKW(RD, WD, Z, W)                                                                                          \
    do {                                                                                                           \
        dim3 g((unsigned)cdiv(A.nslices, SliceGroup<W>::SPB)), t(SliceGroup<W>::THREADS);                          \
        if (e0)                                                                                                    \
            hipExtLaunchKernelGGL((smooth_k<T, B, RD, WD, Z, W>), g, t, 0, s, e0, e1, 0, A.nslices,                \
                                  (const int32_t*)A.off, (const int32_t*)A.rowid, (const int32_t*)A.ci,            \
                                  (const T*)A.v, Dinv, b, xin, d, xout, c1, c2);                                   \
        else                                                                                                       \
            smooth_k<T, B, RD, WD, Z, W><<<g, t, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, Dinv, b, xin, d,    \
                                                        xout, c1, c2);                                             \
    } while (0)
#define SK(RD, WD, Z)                                                                                              \
    do {                                                                                                           \
        if (wps == 16) SKW(RD, WD, Z, 16);                                                                         \
        else if (wps == 8) SKW(RD, WD, Z, 8);                                                                      \
        else if (wps == 4) SKW(RD, WD, Z, 4);                                                                      \
        else if (wps == 2) SKW(RD, WD, Z, 2);                                                                      \
        else SKW(RD, WD, Z, 1);                                                                                    \
    } while (0)
    if (zero) {
        if (wd) SKW(false, true, true, 1); else SKW(false, false, true, 1);
    } else if (rd) {
        if (wd) SK(true, true, false); else SK(true, false, false);
    } else {
        if (wd) SK(false, true, false); else SK(false, false, false);
    }
#undef SK
#undef SKW
    check_launch("smooth_step");
}

template <typename T>
void smooth_step(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, double c1, double c2,
                 bool read_d, bool write_d, bool zero_in, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (A.br) {
        case 1: smooth_dispatch<T, 1>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s, e0, e1); break;
        case 3:
            if (A.rowlane) smooth_rl3<T>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s, e0, e1);
            else smooth_dispatch<T, 3>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s, e0, e1);
            break;
        case 6: smooth_dispatch<T, 6>(A, Dinv, b, xin, d, xout, (T)c1, (T)c2, read_d, write_d, zero_in, s, e0, e1); break;
        default: throw Error(SCR_E_UNIMPLEMENTED, "smooth_step: block size");
    }
}
template void smooth_step<double>(const DSell<double>&, const double*, const double*, const double*, double*, double*,
                                  double, double, bool, bool, bool, hipStream_t, hipEvent_t, hipEvent_t);
template void smooth_step<float>(const DSell<float>&, const float*, const float*, const float*, float*, float*,
                                 double, double, bool, bool, bool, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------- three interleaved columns (1x1 blocks)
// The scalar mesh Laplacian acts on x, y and z alike (Sec. 5.2.2): its products, smoother steps,
// restriction and coarse solve take the three columns of node-interleaved vectors (entry 3 i + c)
// in one pass over the matrix.  Per column every sum is taken in the order of the one-column
// kernels above (same slot order, same slice split, same lane tree), so each column's result is
// bitwise that of the one-column kernel.

// the three-column form of sell_row_dot for 1x1 blocks: the slot's column index and value are
// loaded once and the three x entries of the column gathered together; each column accumulates in
// the slot order of the one-column loop (the same unroll, the same terms)
template <typename T>
__device__ __forceinline__ void sell_row_dot3(int64_t o0, int64_t o1, int lane, const int32_t* __restrict__ ci,
                                              const T* __restrict__ v, const T* __restrict__ x, T (&acc)[3]) {
    acc[0] = acc[1] = acc[2] = 0;
    const int64_t g1 = o1 / SELL_G;
    int64_t g = o0 / SELL_G;
    SellI4 c[2];
    if (g + 2 <= g1) {
        c[0] = sell_gidx(ci, g, lane);
        c[1] = sell_gidx(ci, g + 1, lane);
    }
    for (; g + 2 <= g1; g += 2) {
        T xx[2][SELL_G][3], vv[2][SELL_G];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < SELL_G; ++j)
#pragma unroll
                for (int k = 0; k < 3; ++k) xx[u][j][k] = x[3 * (int64_t)c[u][j] + k];
        SellI4 cn[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) cn[u] = sell_gidx(ci, g + 2 + u < g1 ? g + 2 + u : g1 - 1, lane);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) sell_gvals<T>(v, g + u, lane, vv[u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < SELL_G; ++j)
#pragma unroll
                for (int k = 0; k < 3; ++k) acc[k] += vv[u][j] * xx[u][j][k];
#pragma unroll
        for (int u = 0; u < 2; ++u) c[u] = cn[u];
    }
    for (; g < g1; ++g) {
        const SellI4 cc = sell_gidx(ci, g, lane);
        T vv[SELL_G];
        sell_gvals<T>(v, g, lane, vv);
#pragma unroll
        for (int j = 0; j < SELL_G; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k] += vv[j] * x[3 * (int64_t)cc[j] + k];
    }
}
template <typename T, int MODE, int WPS>
__global__ void __launch_bounds__(SliceGroup<WPS>::THREADS) sell_mv3_k(int64_t nslices, const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ rowid, const int32_t* __restrict__ ci,
                                                  const T* __restrict__ v, const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ y) {
    int wv = threadIdx.x / WAVE;
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * SliceGroup<WPS>::SPB + wv / WPS;
    int lane = threadIdx.x & (WAVE - 1);
    bool live = sl < nslices;
    T acc[3] = {0, 0, 0};
    if (live) {
        int64_t a, e;
        slice_part<WPS, SELL_G>(off[sl], off[sl + 1], wv % WPS, a, e);
        sell_row_dot3<T>(a, e, lane, ci, v, x, acc);
    }
    if (WPS > 1) {
        __shared__ T red[SliceGroup<WPS>::SPB * WPS][3][WAVE];
#pragma unroll
        for (int c = 0; c < 3; ++c) red[wv][c][lane] = acc[c];
        __syncthreads();
        if (wv % WPS != 0) return;
        for (int w = 1; w < WPS; ++w)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += red[wv + w][c][lane];
    }
    if (!live) return;
    int64_t i = rowid[sl * WAVE + lane];
    if (i < 0) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int64_t o = 3 * i + c;
        if (MODE == 0) y[o] = acc[c];
        else if (MODE == 1) y[o] = b[o] - acc[c];
        else if (MODE == 2) y[o] += acc[c];
        else y[o] -= acc[c];
    }
}

template <typename T>
void sell_mv3(const DSell<T>& A, const T* x, const T* b, T* y, int mode, hipStream_t s) {
    if (A.br != 1 || A.bc != 1 || A.rowlane) throw Error(SCR_E_UNIMPLEMENTED, "sell_mv3: 1x1 blocks only");
    if (A.nslices == 0) return;
    int wps = waves_per_slice(A);
#define MV3(W)                                                                                                  \
    {                                                                                                           \
        constexpr int W_ = W;                                                                                   \
        dim3 g((unsigned)cdiv(A.nslices, SliceGroup<W_>::SPB)), th(SliceGroup<W_>::THREADS);                    \
        switch (mode) {                                                                                         \
            case 0: sell_mv3_k<T, 0, W_><<<g, th, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
            case 1: sell_mv3_k<T, 1, W_><<<g, th, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
            case 2: sell_mv3_k<T, 2, W_><<<g, th, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
            default: sell_mv3_k<T, 3, W_><<<g, th, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, x, b, y); break; \
        }                                                                                                       \
    }
    if (wps == 1) MV3(1)
    else if (wps == 2) MV3(2)
    else if (wps == 4) MV3(4)
    else if (wps == 8) MV3(8)
    else MV3(16)
#undef MV3
    check_launch("sell_mv3");
}
template void sell_mv3<double>(const DSell<double>&, const double*, const double*, double*, int, hipStream_t);
template void sell_mv3<float>(const DSell<float>&, const float*, const float*, float*, int, hipStream_t);

// y = R x for 1x1 R (rows of R are long; one row per wavefront, the lane tree of bsrt_mv_k)
template <typename T>
__global__ void __launch_bounds__(256) bsrt_mv3_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  const T* __restrict__ v, const T* __restrict__ x, T* __restrict__ y) {
    int64_t row = xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x / WAVE);
    if (row >= nr) return;
    int lane = threadIdx.x & (WAVE - 1);
    T acc[3] = {0, 0, 0};
    int64_t q0 = rp[row], len = rp[row + 1] - q0;
    for (int64_t j = lane; j < len; j += WAVE) {
        int64_t c = ci[q0 + j];
        const T vv = v[q0 + j];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += vv * x[3 * c + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T sum = wave_sum(acc[k]);
        if (lane == 0) y[3 * row + k] = sum;
    }
}
template <typename T>
void bsrt_mv3(const DBsrT<T>& R, const T* x, T* y, hipStream_t s) {
    if (R.br != 1 || R.bc != 1) throw Error(SCR_E_UNIMPLEMENTED, "bsrt_mv3: 1x1 blocks only");
    int64_t nblk = cdiv(R.nr, 4);
    if (nblk == 0) return;
    bsrt_mv3_k<T><<<nblk, 256, 0, s>>>(R.nr, R.rp, R.ci, R.v, x, y);
    check_launch("bsrt_mv3");
}
template void bsrt_mv3<double>(const DBsrT<double>&, const double*, double*, hipStream_t);
template void bsrt_mv3<float>(const DBsrT<float>&, const float*, float*, hipStream_t);

// one smoothing step on three columns (1x1 blocks): as smooth_k with B = 1, per column
template <typename T, bool RD, bool WD, bool ZERO, int WPS>
__global__ void __launch_bounds__(SliceGroup<WPS>::THREADS) smooth3_k(int64_t nslices, const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ rowid, const int32_t* __restrict__ ci,
                                                 const T* __restrict__ v, const T* __restrict__ Dinv,
                                                 const T* __restrict__ b, const T* __restrict__ xin, T* __restrict__ d,
                                                 T* __restrict__ xout, T c1, T c2) {
    int wv = threadIdx.x / WAVE;
    int64_t sl = xcd_tile(blockIdx.x, gridDim.x) * SliceGroup<WPS>::SPB + wv / WPS;
    bool live = sl < nslices;
    int lane = threadIdx.x & (WAVE - 1);
    T acc[3] = {0, 0, 0};
    if (!ZERO && live) {
        int64_t a, e;
        slice_part<WPS, SELL_G>(off[sl], off[sl + 1], wv % WPS, a, e);
        sell_row_dot3<T>(a, e, lane, ci, v, xin, acc);
    }
    if (WPS > 1) {
        __shared__ T red[SliceGroup<WPS>::SPB * WPS][3][WAVE];
#pragma unroll
        for (int c = 0; c < 3; ++c) red[wv][c][lane] = acc[c];
        __syncthreads();
        if (wv % WPS != 0) return;
        for (int w = 1; w < WPS; ++w)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += red[wv + w][c][lane];
    }
    if (!live) return;
    int64_t i = rowid[sl * WAVE + lane];
    if (i < 0) return;
    const T di = Dinv[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t o = 3 * i + c;
        const T res = b[o] - acc[c];
        T z = 0;
        z += di * res;
        T dn = c2 * z;
        if (RD) dn += c1 * d[o];
        if (WD) d[o] = dn;
        xout[o] = ZERO ? dn : xin[o] + dn;
    }
}

template <typename T>
void smooth_step3(const DSell<T>& A, const T* Dinv, const T* b, const T* xin, T* d, T* xout, double c1, double c2,
                  bool read_d, bool write_d, bool zero_in, hipStream_t s) {
    if (A.br != 1 || A.bc != 1 || A.rowlane) throw Error(SCR_E_UNIMPLEMENTED, "smooth_step3: 1x1 blocks only");
    if (A.nslices == 0) return;
    const T C1 = (T)c1, C2 = (T)c2;
    int wps = zero_in ? 1 : waves_per_slice(A);
#define S3W(RD, WD, Z, W)                                                                                        \
    do {                                                                                                         \
        dim3 g((unsigned)cdiv(A.nslices, SliceGroup<W>::SPB)), th(SliceGroup<W>::THREADS);                        \
        smooth3_k<T, RD, WD, Z, W><<<g, th, 0, s>>>(A.nslices, A.off, A.rowid, A.ci, A.v, Dinv, b, xin, d, xout,  \
                                                   C1, C2);                                                      \
    } while (0)
#define S3(RD, WD, Z)                                                                                            \
    do {                                                                                                         \
        if (wps == 16) S3W(RD, WD, Z, 16);                                                                       \
        else if (wps == 8) S3W(RD, WD, Z, 8);                                                                    \
        else if (wps == 4) S3W(RD, WD, Z, 4);                                                                    \
        else if (wps == 2) S3W(RD, WD, Z, 2);                                                                    \
        else S3W(RD, WD, Z, 1);                                                                                  \
    } while (0)
    if (zero_in) {
        if (write_d) S3W(false, true, true, 1); else S3W(false, false, true, 1);
    } else if (read_d) {
        if (write_d) S3(true, true, false); else S3(true, false, false);
    } else {
        if (write_d) S3(false, true, false); else S3(false, false, false);
    }
#undef S3
#undef S3W
    check_launch("smooth_step3");
}
template void smooth_step3<double>(const DSell<double>&, const double*, const double*, const double*, double*,
                                   double*, double, double, bool, bool, bool, hipStream_t);
template void smooth_step3<float>(const DSell<float>&, const float*, const float*, const float*, float*, float*,
                                  double, double, bool, bool, bool, hipStream_t);

// x = M b on three columns (the lane tree of dense_mv_k, per column)
template <typename T>
__global__ void __launch_bounds__(256) dense_mv3_k(int64_t n, const double* __restrict__ M, const T* __restrict__ b,
                                                   T* __restrict__ x) {
    int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (row >= n) return;
    int lane = threadIdx.x & (WAVE - 1);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t c = lane; c < n; c += WAVE) {
        const double m = M[row * n + c];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += m * (double)b[3 * c + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double sum = wave_sum(acc[k]);
        if (lane == 0) x[3 * row + k] = (T)sum;
    }
}
template <typename T>
void dense_mv3(int64_t n, const double* M, const T* b, T* x, hipStream_t s) {
    if (n <= 0) return;
    dense_mv3_k<T><<<cdiv(n, 4), 256, 0, s>>>(n, M, b, x);
    check_launch("dense_mv3");
}
template void dense_mv3<double>(int64_t, const double*, const double*, double*, hipStream_t);
template void dense_mv3<float>(int64_t, const double*, const float*, float*, hipStream_t);

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
// One wavefront per row (lane l checks entries lo + l, lo + l + 64, ...); the bits found are OR-ed
// over the wavefront and raised by one atomic.
__global__ void __launch_bounds__(256) validate_k(int64_t nr, int bs, int64_t nnzb, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                  int* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    if (i >= nr) return;
    const int lane = threadIdx.x & (WAVE - 1);
    int f = 0;
    const int64_t lo = rp[i], hi = rp[i + 1];
    if (i == 0 && lo != 0) f |= 1;
    if (i == nr - 1 && hi != nnzb) f |= 1;
    if (lo < 0 || hi > nnzb || lo > hi) {
        if (lane == 0) atomicOr(flags, f | 1);
        return;
    }
    bool diag = false;
    const int bb = bs * bs;
    const int nd = bs == 4 ? 3 : bs;   // the velocity diagonal (diag(A)) must be nonzero
    for (int64_t q = lo + lane; q < hi; q += WAVE) {
        const int64_t c = ci[q];
        if (c < 0 || c >= nr) { f |= 2; continue; }
        const int64_t pc = q > lo ? ci[q - 1] : -1;   // an out-of-range neighbour is reported as such
        if (pc >= 0 && pc < nr && c <= pc) f |= 4;
        for (int e = 0; e < bb; ++e)
            if (!isfinite(v[q * bb + e])) f |= 16;
        if (c == i) {
            diag = true;
            for (int k = 0; k < nd; ++k)
                if (v[q * bb + k * bs + k] == 0.0) f |= 32;
        }
    }
    if (!__any(diag)) f |= 8;
    for (int o = WAVE / 2; o > 0; o >>= 1) f |= __shfl_xor(f, o, WAVE);
    if (lane == 0 && f) atomicOr(flags, f);
}

int validate_bsr(int64_t nr, int bs, int64_t nnzb, const int32_t* rp, const int32_t* ci, const double* v, Arena& ar,
                 hipStream_t s) {
    int* flags = ar.make<int>(1);
    zero_dev(flags, sizeof(int), s);
    if (nr > 0) validate_k<<<cdiv(nr, 256 / WAVE), 256, 0, s>>>(nr, bs, nnzb, rp, ci, v, flags);
    check_launch("validate");
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(flags);
    return h;
}

}  // namespace scr
