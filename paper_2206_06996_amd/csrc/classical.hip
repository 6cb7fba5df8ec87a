// classical.hip -- classical AMG on the device with the settings of the paper's table of
// BoomerAMG options (Sec. 5.2): classical strength (threshold 0.5), HMIS coarsening, extended+i
// interpolation truncated at 0.3 with at most 5 entries per row, aggressive (two-stage) coarsening
// on the first levels, hybrid Gauss-Seidel smoothing (l1 form by default), V-cycle with Galerkin
// coarse operators and a direct coarsest solve.
//
// Mapping to the chip.  HMIS's per-processor first pass (Ruge-Stueben) runs with one workgroup
// per domain of 256 consecutive rows: the measures and states live in LDS, each step picks the
// domain's largest measure by a workgroup reduction, and the C/F updates are LDS integer atomics
// (order-free, so the result is that of the sequential pass).  The PMIS rounds and extended+i are
// row-parallel.  Hybrid Gauss-Seidel gives each workgroup a domain of 64 rows: its wavefronts
// first gather, with no dependency between rows, every row's previous-iterate sum and its
// couplings to earlier rows of the sweep into LDS; one wavefront then sweeps the domain with one
// lane per row, each new value broadcast to the later lanes, so no global load sits in the chain.
// Interpolation weights, their truncation and the Galerkin products are evaluated in the
// definitions' order without fused multiply-adds (this file is built with -ffp-contract=off), so
// every level's split, pattern and values are those of a sequential evaluation.
#include <algorithm>
#include <memory>
#include <type_traits>

#include "solver.h"

namespace scr {
namespace {

constexpr int HMIS_DOM = 256;      // rows per HMIS domain (one workgroup)
constexpr int GS_DOM = 64;         // rows per hybrid Gauss-Seidel domain (one workgroup; one lane per row in its sequential phase)
constexpr int8_t ST_U = 0, ST_C = 1, ST_F = 2, ST_NEWF = 3;

// ------------------------------------------------------------------ set-up kernels
// scalar rows of a b x b block matrix: row b i + r holds, block by block, the entries of row r
__global__ void to_scalar_k(int64_t nb, int b, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ v, int32_t* __restrict__ srp, int32_t* __restrict__ sci,
                            double* __restrict__ sv, uint8_t* __restrict__ func) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int32_t q0 = rp[i], len = rp[i + 1] - q0;
    for (int r = 0; r < b; ++r) {
        const int64_t row = (int64_t)b * i + r;
        int64_t p = (int64_t)b * b * q0 + (int64_t)r * b * len;
        srp[row] = (int32_t)p;
        func[row] = (uint8_t)r;
        for (int32_t q = q0; q < q0 + len; ++q)
            for (int c = 0; c < b; ++c) {
                sci[p] = ci[q] * b + c;
                sv[p] = v[(int64_t)q * b * b + r * b + c];
                ++p;
            }
    }
    if (i == nb - 1) srp[(int64_t)b * nb] = (int32_t)((int64_t)b * b * rp[nb]);
}

__device__ __forceinline__ int32_t find_sorted_dev(const int32_t* __restrict__ v, int32_t lo, int32_t hi, int32_t key) {
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (v[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// tmap[q] = position of (j, i) for q = (i, j); err if the pattern is not structurally symmetric
__global__ void tmap_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       int32_t* __restrict__ tmap, int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int32_t j = ci[q];
        const int32_t t = find_sorted_dev(ci, rp[j], rp[j + 1], (int32_t)i);
        if (t < rp[j + 1] && ci[t] == i) tmap[q] = t;
        else { tmap[q] = -1; *err = 1; }
    }
}

// classical strength within a function: -s a_ij >= theta max_k(-s a_ik), s = sign(a_ii)
__global__ void cl_strength_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const double* __restrict__ v, const uint8_t* __restrict__ func, double theta,
                              uint8_t* __restrict__ S) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    double aii = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        if (ci[q] == i) aii = v[q];
    const double sg = aii < 0.0 ? -1.0 : 1.0;
    bool have = false;
    double m = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int32_t j = ci[q];
        if (j == i || func[j] != func[i]) continue;
        const double x = -sg * v[q];
        if (!have || x > m) { m = x; have = true; }
    }
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int32_t j = ci[q];
        uint8_t f = 0;
        if (j != i && func[j] == func[i] && have && m > 0.0) f = (uint8_t)(-sg * v[q] >= theta * m);
        S[q] = f;
    }
}

// Ruge-Stueben first pass inside one domain of HMIS_DOM rows per workgroup (writes first[i]:
// 1 = C, -1 = F).  One C point per step: the undecided point of largest measure, lowest row on ties.
__global__ void __launch_bounds__(HMIS_DOM) hmis_first_k(int64_t nr, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const uint8_t* __restrict__ S,
                                                         const int32_t* __restrict__ tmap, int8_t* __restrict__ first) {
    __shared__ int lam[HMIS_DOM];
    __shared__ int8_t st[HMIS_DOM];
    __shared__ long long red[HMIS_DOM / WAVE];
    const int t = threadIdx.x;
    const int64_t d0 = (int64_t)blockIdx.x * HMIS_DOM;
    const int64_t d1 = d0 + HMIS_DOM < nr ? d0 + HMIS_DOM : nr;
    const int64_t i = d0 + t;
    const bool live = i < d1;
    if (live) {
        int l = 0, dep = 0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int64_t j = ci[q];
            if (j < d0 || j >= d1) continue;
            l += S[tmap[q]];
            dep += S[q];
        }
        lam[t] = l;
        st[t] = (l == 0 && dep == 0) ? ST_F : ST_U;
    } else {
        lam[t] = 0;
        st[t] = ST_F;
    }
    __syncthreads();
    for (;;) {
        // key: measure (biased positive) then 255 - t, so the maximum is the largest measure, lowest t
        long long key = st[t] == ST_U ? (((long long)lam[t] + (1LL << 30)) << 8) | (long long)(HMIS_DOM - 1 - t) : -1;
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            long long w = __shfl_xor(key, o, WAVE);
            key = w > key ? w : key;
        }
        if ((t & (WAVE - 1)) == 0) red[t / WAVE] = key;
        __syncthreads();
        long long best = red[0];
        for (int w = 1; w < HMIS_DOM / WAVE; ++w) best = red[w] > best ? red[w] : best;
        __syncthreads();
        if (best < 0) break;
        const int c = HMIS_DOM - 1 - (int)(best & 0xFF);
        const int64_t cr = d0 + c;
        if (t == c) st[c] = ST_C;
        __syncthreads();
        // the domain's undecided points that depend on c become F
        for (int32_t q = rp[cr] + t; q < rp[cr + 1]; q += HMIS_DOM) {
            const int64_t j = ci[q];
            if (j >= d0 && j < d1 && st[j - d0] == ST_U && S[tmap[q]]) st[j - d0] = ST_NEWF;
        }
        __syncthreads();
        // the undecided points c depends on lose one unit of measure
        for (int32_t q = rp[cr] + t; q < rp[cr + 1]; q += HMIS_DOM) {
            const int64_t j = ci[q];
            if (j >= d0 && j < d1 && st[j - d0] == ST_U && S[q]) atomicSub(&lam[j - d0], 1);
        }
        // the undecided points each new F point depends on gain one
        if (live && st[t] == ST_NEWF)
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
                const int64_t k = ci[q];
                if (k >= d0 && k < d1 && st[k - d0] == ST_U && S[q]) atomicAdd(&lam[k - d0], 1);
            }
        __syncthreads();
        if (st[t] == ST_NEWF) st[t] = ST_F;
        __syncthreads();
    }
    if (live) first[i] = st[t] == ST_C ? 1 : -1;
}

__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

// PMIS start: measure |S^T_i| + u_i; C for first-pass C points whose strong connections stay in
// their domain; F for points that influence nobody; the rest undecided
__global__ void pmis_init_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const uint8_t* __restrict__ S, const int32_t* __restrict__ tmap,
                            const int8_t* __restrict__ first, uint64_t seed, int level, double* __restrict__ w,
                            int8_t* __restrict__ st, uint8_t* __restrict__ isnew) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const int64_t dm = i / HMIS_DOM;
    bool interior = true;
    int nst = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const uint8_t sT = S[tmap[q]];
        nst += sT;
        if ((S[q] || sT) && (int64_t)ci[q] / HMIS_DOM != dm) interior = false;
    }
    const uint64_t h = splitmix(seed ^ ((uint64_t)level << 56) ^ ((uint64_t)i * 0x9E6C63D0676A9A99ULL));
    w[i] = (double)nst + (double)(h >> 11) * 0x1.0p-53;
    int8_t s;
    if (first[i] == 1 && interior) s = ST_C;
    else s = nst == 0 ? ST_F : ST_U;
    st[i] = s;
    isnew[i] = s == ST_C;
}

// undecided points that depend on a C point of the previous round become F; counts the undecided
__global__ void pmis_f_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const uint8_t* __restrict__ S, const uint8_t* __restrict__ isnew, const int8_t* __restrict__ st,
                         int8_t* __restrict__ out, int* __restrict__ und) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int u = 0;
    if (i < nr) {
        int8_t s = st[i];
        if (s == ST_U)
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
                if (S[q] && isnew[ci[q]]) { s = ST_F; break; }
        out[i] = s;
        u = s == ST_U;
    }
    // one atomic per wavefront
    for (int o = WAVE / 2; o > 0; o >>= 1) u += __shfl_xor(u, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && u) atomicAdd(und, u);
}

// undecided points whose measure beats every undecided strong neighbour's (either direction)
__global__ void pmis_c_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const uint8_t* __restrict__ S, const int32_t* __restrict__ tmap, const double* __restrict__ w,
                         const int8_t* __restrict__ st, uint8_t* __restrict__ isnew) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    bool best = st[i] == ST_U;
    for (int32_t q = rp[i]; q < rp[i + 1] && best; ++q) {
        const int64_t j = ci[q];
        if (j == i || st[j] != ST_U || !(S[q] || S[tmap[q]])) continue;
        if (!(w[i] > w[j] || (w[i] == w[j] && i < j))) best = false;
    }
    isnew[i] = best;
}

__global__ void pmis_apply_k(int64_t nr, const uint8_t* __restrict__ isnew, int8_t* __restrict__ st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr && isnew[i]) st[i] = ST_C;
}

__global__ void cflag_k(int64_t nr, const int8_t* __restrict__ st, int32_t* __restrict__ f) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) f[i] = st[i] == ST_C;
}

__global__ void cidx_k(int64_t nr, const int8_t* __restrict__ st, const int32_t* __restrict__ rank,
                       int32_t* __restrict__ cidx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) cidx[i] = st[i] == ST_C ? rank[i] : -1;
}

__global__ void coarse_func_k(int64_t nr, const int32_t* __restrict__ cidx, const uint8_t* __restrict__ func,
                              uint8_t* __restrict__ fc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr && cidx[i] >= 0) fc[cidx[i]] = func[i];
}

// upper bound of |C^_i| (1 for C points)
__global__ void extpi_cap_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const uint8_t* __restrict__ S, const int32_t* __restrict__ cidx, int32_t* __restrict__ cap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    if (cidx[i] >= 0) { cap[i] = 1; return; }
    int64_t c = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        if (!S[q]) continue;
        const int32_t j = ci[q];
        c += cidx[j] >= 0 ? 1 : rp[j + 1] - rp[j];
    }
    cap[i] = (int32_t)(c < INT32_MAX ? c : INT32_MAX);
}

__device__ __forceinline__ bool opposite(double a, double d) { return (a > 0.0 && d < 0.0) || (a < 0.0 && d > 0.0); }

__device__ void heap_sift(int32_t* a, int64_t n, int64_t r) {
    for (;;) {
        int64_t c = 2 * r + 1;
        if (c >= n) return;
        if (c + 1 < n && a[c + 1] > a[c]) ++c;
        if (a[r] >= a[c]) return;
        int32_t t = a[r]; a[r] = a[c]; a[c] = t;
        r = c;
    }
}
__device__ void heap_sort(int32_t* a, int64_t n) {
    for (int64_t r = n / 2 - 1; r >= 0; --r) heap_sift(a, n, r);
    for (int64_t e = n - 1; e > 0; --e) {
        int32_t t = a[0]; a[0] = a[e]; a[e] = t;
        heap_sift(a, e, 0);
    }
}
__device__ __forceinline__ int64_t in_hat(const int32_t* hat, int64_t m, int32_t key) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (hat[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < m && hat[lo] == key) ? lo : -1;
}

// Truncation of one interpolation row (columns ascending, non-negative): entries below trunc times
// the largest magnitude dropped (and exact zeros), then all but the pmax largest (lower column on
// ties), then the kept entries scaled to the row's original sum.  Compacts in place; returns the
// kept count.  The sums run in column order, as in the definition.
__device__ int64_t truncate_seg(int32_t* col, double* w, int64_t m, double trunc, int pmax) {
    double mx = 0.0, all = 0.0;
    for (int64_t t = 0; t < m; ++t) {
        all = all + w[t];
        if (fabs(w[t]) > mx) mx = fabs(w[t]);
    }
    int64_t k = 0;
    for (int64_t t = 0; t < m; ++t)
        if (w[t] != 0.0 && fabs(w[t]) >= trunc * mx) { col[k] = col[t]; w[k] = w[t]; ++k; }
    if (k > pmax) {
        // the pmax largest magnitudes, lower column first on ties: mark them by negating the column
        for (int s = 0; s < pmax; ++s) {
            int64_t b = -1;
            for (int64_t t = 0; t < k; ++t) {
                if (col[t] < 0) continue;
                if (b < 0 || fabs(w[t]) > fabs(w[b])) b = t;
            }
            col[b] = -1 - col[b];
        }
        int64_t k2 = 0;
        for (int64_t t = 0; t < k; ++t)
            if (col[t] < 0) { col[k2] = -1 - col[t]; w[k2] = w[t]; ++k2; }
        k = k2;
    }
    double kept = 0.0;
    for (int64_t t = 0; t < k; ++t) kept = kept + w[t];
    if (kept != 0.0) {
        const double sc = all / kept;
        for (int64_t t = 0; t < k; ++t) w[t] = w[t] * sc;
    }
    return k;
}

// extended+i row i into its scratch segment [off_i, off_i + cap_i): the kept coarse columns
// (ascending) and weights at its front, their count in cnt[i]
__global__ void extpi_row_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ v, const uint8_t* __restrict__ func,
                            const uint8_t* __restrict__ S, const int32_t* __restrict__ cidx,
                            const int32_t* __restrict__ off, double trunc, int pmax, int32_t* __restrict__ hcol,
                            double* __restrict__ hw, int32_t* __restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    int32_t* hat = hcol + off[i];
    double* w = hw + off[i];
    if (cidx[i] >= 0) {
        hat[0] = cidx[i];
        w[0] = 1.0;
        cnt[i] = 1;
        return;
    }
    // C^_i: strong C neighbours and the strong C neighbours of strong F neighbours (sorted, unique)
    int64_t m = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        if (!S[q]) continue;
        const int32_t j = ci[q];
        if (cidx[j] >= 0) { hat[m++] = j; continue; }
        for (int32_t r = rp[j]; r < rp[j + 1]; ++r)
            if (S[r] && cidx[ci[r]] >= 0) hat[m++] = ci[r];
    }
    heap_sort(hat, m);
    int64_t u = 0;
    for (int64_t t = 0; t < m; ++t)
        if (u == 0 || hat[t] != hat[u - 1]) hat[u++] = hat[t];
    m = u;
    double diag = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        if (ci[q] == i) diag = v[q];
    for (int64_t t = 0; t < m; ++t) w[t] = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int32_t n = ci[q];
        if (n == i || func[n] != func[i]) continue;
        const int64_t p = in_hat(hat, m, n);
        if (p >= 0) { w[p] = w[p] + v[q]; continue; }
        if (S[q] && cidx[n] < 0) {
            double ann = 0.0, den = 0.0;
            for (int32_t r = rp[n]; r < rp[n + 1]; ++r)
                if (ci[r] == n) ann = v[r];
            for (int32_t r = rp[n]; r < rp[n + 1]; ++r) {
                const int32_t l = ci[r];
                if ((l == i || in_hat(hat, m, l) >= 0) && opposite(v[r], ann)) den = den + v[r];
            }
            if (den == 0.0) { diag = diag + v[q]; continue; }
            for (int32_t r = rp[n]; r < rp[n + 1]; ++r) {
                const int32_t l = ci[r];
                if (!opposite(v[r], ann)) continue;
                const double x = (v[q] * v[r]) / den;
                if (l == i) diag = diag + x;
                else {
                    const int64_t pl = in_hat(hat, m, l);
                    if (pl >= 0) w[pl] = w[pl] + x;
                }
            }
            continue;
        }
        diag = diag + v[q];
    }
    if (m == 0 || diag == 0.0) { cnt[i] = 0; return; }
    for (int64_t t = 0; t < m; ++t) w[t] = -w[t] / diag;
    const int64_t k = truncate_seg(hat, w, m, trunc, pmax);
    for (int64_t t = 0; t < k; ++t) hat[t] = cidx[hat[t]];
    cnt[i] = (int32_t)k;
}

__global__ void extpi_fill_k(int64_t nr, const int32_t* __restrict__ off, const int32_t* __restrict__ hcol,
                             const double* __restrict__ hw, const int32_t* __restrict__ prp, int32_t* __restrict__ pci,
                             double* __restrict__ pv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const int32_t n = prp[i + 1] - prp[i];
    for (int32_t t = 0; t < n; ++t) {
        pci[prp[i] + t] = hcol[off[i] + t];
        pv[prp[i] + t] = hw[off[i] + t];
    }
}

// truncation of every row of a product P = P1 P2 in place (kept entries at the front of each row)
__global__ void trunc_rows_k(int64_t nr, const int32_t* __restrict__ rp, int32_t* __restrict__ ci,
                             double* __restrict__ v, double trunc, int pmax, int32_t* __restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    cnt[i] = (int32_t)truncate_seg(ci + rp[i], v + rp[i], rp[i + 1] - rp[i], trunc, pmax);
}

// ---- aggressive coarsening: the second-stage graph on the first-stage C points
__global__ void fine_of_k(int64_t nr, const int32_t* __restrict__ c1, int32_t* __restrict__ fine_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr && c1[i] >= 0) fine_of[c1[i]] = (int32_t)i;
}
// upper bound of the out-edges of C point a: one per strong dependency and its row
__global__ void ss_cap_k(int64_t n1, const int32_t* __restrict__ fine_of, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ ci, const uint8_t* __restrict__ S, int32_t* __restrict__ cap) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n1) return;
    const int64_t i = fine_of[a];
    int64_t c = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        if (S[q]) c += 1 + (rp[ci[q] + 1] - rp[ci[q]]);
    cap[a] = (int32_t)(c < INT32_MAX ? c : INT32_MAX);
}
// the out-edges of a (C points reached by one or two strong dependencies), sorted and unique
__global__ void ss_out_k(int64_t n1, const int32_t* __restrict__ fine_of, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ ci, const uint8_t* __restrict__ S, const int32_t* __restrict__ c1,
                         const int32_t* __restrict__ off, int32_t* __restrict__ buf, int32_t* __restrict__ no) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n1) return;
    const int64_t i = fine_of[a];
    int32_t* e = buf + off[a];
    int64_t m = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        if (!S[q]) continue;
        const int32_t k = ci[q];
        if (c1[k] >= 0 && k != i) e[m++] = c1[k];
        for (int32_t r = rp[k]; r < rp[k + 1]; ++r)
            if (S[r] && c1[ci[r]] >= 0 && ci[r] != i) e[m++] = c1[ci[r]];
    }
    heap_sort(e, m);
    int64_t u = 0;
    for (int64_t t = 0; t < m; ++t)
        if (u == 0 || e[t] != e[u - 1]) e[u++] = e[t];
    no[a] = (int32_t)u;
}
__global__ void ss_indeg_k(int64_t n1, const int32_t* __restrict__ off, const int32_t* __restrict__ buf,
                           const int32_t* __restrict__ no, int32_t* __restrict__ nin) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n1) return;
    for (int32_t t = 0; t < no[a]; ++t) atomicAdd(&nin[buf[off[a] + t]], 1);
}
__global__ void ss_in_fill_k(int64_t n1, const int32_t* __restrict__ off, const int32_t* __restrict__ buf,
                             const int32_t* __restrict__ no, const int32_t* __restrict__ inoff, int32_t* __restrict__ cur,
                             int32_t* __restrict__ inbuf) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n1) return;
    for (int32_t t = 0; t < no[a]; ++t) {
        const int32_t b = buf[off[a] + t];
        inbuf[inoff[b] + atomicAdd(&cur[b], 1)] = (int32_t)a;
    }
}
// the in-lists sorted (their fill order came from atomics)
__global__ void ss_in_sort_k(int64_t n1, const int32_t* __restrict__ inoff, const int32_t* __restrict__ nin,
                             int32_t* __restrict__ inbuf) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n1) heap_sort(inbuf + inoff[b], nin[b]);
}
// row a of the symmetric pattern: the merge of its out- and in-lists, flag = out-edge
// (FILL = false: count only)
template <bool FILL>
__global__ void ss_merge_k(int64_t n1, const int32_t* __restrict__ off, const int32_t* __restrict__ buf,
                           const int32_t* __restrict__ no, const int32_t* __restrict__ inoff,
                           const int32_t* __restrict__ inbuf, const int32_t* __restrict__ nin,
                           const int32_t* __restrict__ rp2, int32_t* __restrict__ ci2, uint8_t* __restrict__ f2,
                           int32_t* __restrict__ cnt) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n1) return;
    const int32_t* o = buf + off[a];
    const int32_t* in = inbuf + inoff[a];
    int32_t x = 0, y = 0, p = 0;
    while (x < no[a] || y < nin[a]) {
        const int32_t cx = x < no[a] ? o[x] : INT32_MAX, cy = y < nin[a] ? in[y] : INT32_MAX;
        const int32_t c = cx < cy ? cx : cy;
        if (FILL) {
            ci2[rp2[a] + p] = c;
            f2[rp2[a] + p] = cx == c;
        }
        if (cx == c) ++x;
        if (cy == c) ++y;
        ++p;
    }
    if (!FILL) cnt[a] = p;
}
// coarse index of the level: the second-stage index of the first-stage C points that stayed C
__global__ void agg_compose_k(int64_t nr, const int32_t* __restrict__ c1, const int32_t* __restrict__ c2,
                              int32_t* __restrict__ agg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) agg[i] = c1[i] >= 0 ? c2[c1[i]] : -1;
}

// ------------------------------------------------------------------ hybrid Gauss-Seidel
// l1 form of the sweep's diagonal: ell_i = s sum |a_ij| over the columns outside row i's domain
// of GS_DOM rows (s = sign(a_ii), column order), dinv_i = 1 / (a_ii + ell_i)
__global__ void l1_diag_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ v, double* __restrict__ ell, double* __restrict__ dinv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    double aii = 0.0, e = 0.0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int64_t j = ci[q];
        if (j == i) aii = v[q];
        else if (j / GS_DOM != i / GS_DOM) e = e + fabs(v[q]);
    }
    ell[i] = aii < 0.0 ? -e : e;
    dinv[i] = 1.0 / (aii + ell[i]);
}

// One sweep: x_i = (b_i - sum_{j != i} a_ij x~_j + ell_i xold_i) dinv_i, x~_j new for rows of the
// same domain already swept (forward: j < i; backward: j > i), else the previous iterate xold
// (nullptr: 0); ell nullptr and dinv = 1 / a_ii for the plain sweep, the l1 terms otherwise.
// NC node-interleaved columns (entry NC i + c).  One workgroup per domain of GS_DOM rows, in two
// phases so that no load waits in the sweep's chain of dependencies:
//  1. every row of the domain (GS_W wavefronts, 8 lanes per row, GS_RB rows per lane group and GS_U
//     entries per lane in flight; no dependency between rows): its sum over the couplings that take
//     the previous iterate, into LDS, and its couplings to rows earlier in the sweep (the fresh
//     ones) into LDS as the strictly lower triangle in sweep order, packed by columns;
//  2. the first wavefront, over the sweep positions q: lane q forms its new value, it is broadcast,
//     and every later position subtracts its coupling to it (the fresh part of each row's sum, in
//     sweep order).
constexpr int GS_TRI = GS_DOM * (GS_DOM - 1) / 2;
constexpr int GS_W = 8;             // wavefronts per domain in the first phase
constexpr int GS_U = 8;             // row entries per lane in flight in the first phase
constexpr int GS_RB = 1;            // rows per lane group in flight in the first phase
static_assert(GS_DOM == WAVE, "one lane per row of a domain in the second phase");
static_assert(GS_W * 8 * GS_RB == GS_DOM, "the first phase covers the domain in one pass");

// slot of the coupling of sweep position p to position q < p (column-packed strict lower triangle)
__device__ __forceinline__ int gs_tri(int p, int q) { return (GS_DOM - 1) * q - q * (q - 1) / 2 + (p - q - 1); }

__device__ __forceinline__ double readlane_t(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_t(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <typename T, int NC, bool BWD>
__global__ void __launch_bounds__(GS_W * WAVE) hgs_k(int64_t nr, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                   const T* __restrict__ dinv, const T* __restrict__ ell,
                                                   const T* __restrict__ b, const T* __restrict__ xold,
                                                   T* __restrict__ x) {
    __shared__ T F[GS_TRI];
    __shared__ T so_sh[NC][GS_DOM];
    const int wv = threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t lo = xcd_tile(blockIdx.x, gridDim.x) * GS_DOM;     // the grid covers the rows exactly
    const int64_t hi = lo + GS_DOM < nr ? lo + GS_DOM : nr;
    const int n = (int)(hi - lo);
    for (int e = threadIdx.x; e < GS_TRI; e += GS_W * WAVE) F[e] = T(0);
    __syncthreads();
    // phase 1: wavefront wv takes positions 8 (GS_RB wv + r) + grp, r < GS_RB
    const int grp = lane >> 3, gl = lane & 7;
    const int64_t il = BWD ? hi - 1 - lane : lo + lane;
    const int32_t rs = lane < n ? rp[il] : 0, re = lane < n ? rp[il + 1] : 0;
    int tt[GS_RB];
    int32_t qs[GS_RB], qe[GS_RB];
    int64_t ii[GS_RB];
    int32_t len = 0;
#pragma unroll
    for (int r = 0; r < GS_RB; ++r) {
        tt[r] = 8 * (GS_RB * wv + r) + grp;
        qs[r] = __shfl(rs, tt[r], WAVE);
        qe[r] = __shfl(re, tt[r], WAVE);
        ii[r] = BWD ? hi - 1 - tt[r] : lo + tt[r];
        len = qe[r] - qs[r] > len ? qe[r] - qs[r] : len;
    }
    T acc[GS_RB][NC];
#pragma unroll
    for (int r = 0; r < GS_RB; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = T(0);
    // every load of a step is issued before any is used (the index is clamped to the row's last
    // entry, or to entry 0 for a row with none, so that the loads need no branch)
    for (int32_t o = gl; o < len; o += 8 * GS_U) {
        int32_t jj[GS_RB][GS_U];
        T aa[GS_RB][GS_U];
#pragma unroll
        for (int r = 0; r < GS_RB; ++r)
#pragma unroll
            for (int u = 0; u < GS_U; ++u) {
                const int32_t q = qs[r] + o + 8 * u;
                const int32_t qq = q < qe[r] ? q : (qe[r] > qs[r] ? qe[r] - 1 : 0);
                jj[r][u] = ci[qq];
                aa[r][u] = v[qq];
            }
        T xx[GS_RB][GS_U][NC];
        bool old[GS_RB][GS_U], fresh[GS_RB][GS_U];
        int pjs[GS_RB][GS_U];
#pragma unroll
        for (int r = 0; r < GS_RB; ++r)
#pragma unroll
            for (int u = 0; u < GS_U; ++u) {
                const bool real = qs[r] + o + 8 * u < qe[r];
                const int64_t j = jj[r][u];
                const bool in_dom = j >= lo && j < hi;
                pjs[r][u] = in_dom ? (BWD ? (int)(hi - 1 - j) : (int)(j - lo)) : 0;
                fresh[r][u] = real && in_dom && pjs[r][u] < tt[r];
                old[r][u] = real && !fresh[r][u] && j != ii[r];
                const int64_t jc = old[r][u] ? j : lo;
#pragma unroll
                for (int c = 0; c < NC; ++c) xx[r][u][c] = xold != nullptr ? xold[NC * jc + c] : T(0);
            }
#pragma unroll
        for (int r = 0; r < GS_RB; ++r)
#pragma unroll
            for (int u = 0; u < GS_U; ++u) {
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[r][c] += old[r][u] ? aa[r][u] * xx[r][u][c] : T(0);
                if (fresh[r][u]) F[gs_tri(tt[r], pjs[r][u])] = aa[r][u];
            }
    }
#pragma unroll
    for (int r = 0; r < GS_RB; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            T s = acc[r][c];
#pragma unroll
            for (int w = 1; w < 8; w <<= 1) s += __shfl_xor(s, w, WAVE);
            if (gl == 0) so_sh[c][tt[r]] = s;
        }
    __syncthreads();
    if (wv != 0) return;
    // phase 2 (first wavefront): the row at sweep position `lane`
    const bool own = lane < n;
    const T dv = own ? dinv[il] : T(0);
    const T ev = (own && ell != nullptr && xold != nullptr) ? ell[il] : T(0);
    T r[NC], xn[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        r[c] = own ? b[NC * il + c] - so_sh[c][lane] : T(0);
        if (own && ell != nullptr && xold != nullptr) r[c] = r[c] + ev * xold[NC * il + c];
        xn[c] = T(0);
    }
    for (int q = 0; q < n; ++q) {
        const T f = (lane > q && lane < n) ? F[gs_tri(lane, q)] : T(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (lane == q) xn[c] = r[c] * dv;
            const T xq = readlane_t(xn[c], q);
            r[c] = r[c] - f * xq;
        }
    }
    if (own) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[NC * il + c] = xn[c];
    }
}

// v: the values of A (pattern rp, ci) in T
template <typename T, int NC>
void hgs(const DBsr& A, const T* v, const T* Dinv, const T* ell, const T* b, const T* xold, T* x, bool backward,
         hipStream_t s) {
    const unsigned g = (unsigned)cdiv(A.nr, GS_DOM);     // one workgroup per domain
    if (!g) return;
    if (backward) hgs_k<T, NC, true><<<g, GS_W * WAVE, 0, s>>>(A.nr, A.rp, A.ci, v, Dinv, ell, b, xold, x);
    else hgs_k<T, NC, false><<<g, GS_W * WAVE, 0, s>>>(A.nr, A.rp, A.ci, v, Dinv, ell, b, xold, x);
    check_launch("hybrid_gs");
}

// ------------------------------------------------------------------ hierarchy
class ClassicalBase : public Hierarchy {
   public:
    DBsr pattern0;                   // the block pattern of A0 (no values), for amg_update
    virtual void prepare(Arena& a, hipStream_t s) = 0;
    virtual void release_solve(Arena& a) = 0;
};

// the solve-phase copies in T: FP64, or FP32 for the mixed forms (the V-cycle on FP32 vectors with
// FP32 copies of every level's matrix, diagonal and l1 terms; the coarsest solve with the FP64
// inverse)
template <typename T>
class ClassicalHier : public ClassicalBase {
   public:
    struct LS {
        DSell<T> A, P;
        DBsrT<T> R;
        const T *av = nullptr, *dinv = nullptr, *ell = nullptr;   // what the sweeps read
        T *own_av = nullptr, *own_dinv = nullptr, *own_ell = nullptr;   // FP32 copies (owned)
        T *b = nullptr, *x = nullptr, *w = nullptr, *r = nullptr;
        T *b3 = nullptr, *x3 = nullptr, *w3 = nullptr, *r3 = nullptr;
    };
    std::vector<LS> S;

    void prepare(Arena& a, hipStream_t s) override {
        S.resize(L.size());
        for (size_t l = 0; l < L.size(); ++l) {
            LevelSetup& ls = L[l];
            LS& q = S[l];
            const int64_t n = ls.A.nr;
            q.b = a.make<T>(n); q.x = a.make<T>(n);
            if (three) { q.b3 = a.make<T>(3 * n); q.x3 = a.make<T>(3 * n); }
            if (l + 1 == L.size()) continue;
            q.A = sell_from_bsr<T>(ls.A, a, s);
            q.P = sell_from_bsr<T>(ls.P, a, s);
            q.R = bsrt_from_bsr<T>(ls.R, a, s);
            if constexpr (std::is_same<T, double>::value) {
                q.av = ls.A.v; q.dinv = ls.Dinv; q.ell = ls.ell;
            } else {
                q.own_av = a.make<T>(ls.A.nnzb + 1);
                cast_d2f(ls.A.v, q.own_av, ls.A.nnzb, s);
                q.own_dinv = a.make<T>(n);
                cast_d2f(ls.Dinv, q.own_dinv, n, s);
                if (ls.ell) {
                    q.own_ell = a.make<T>(n);
                    cast_d2f(ls.ell, q.own_ell, n, s);
                }
                q.av = q.own_av; q.dinv = q.own_dinv; q.ell = q.own_ell;
            }
            q.w = a.make<T>(n); q.r = a.make<T>(n);
            if (three) { q.w3 = a.make<T>(3 * n); q.r3 = a.make<T>(3 * n); }
        }
    }
    void release_solve(Arena& a) override {
        for (auto& q : S) {
            sell_free(q.A, a);
            sell_free(q.P, a);
            a.free(q.R.v);
            for (T* p : {q.own_av, q.own_dinv, q.own_ell, q.b, q.x, q.w, q.r, q.b3, q.x3, q.w3, q.r3}) a.free(p);
        }
        S.clear();
    }
    void refresh(Arena& a, hipStream_t s) override {
        release_solve(a);
        prepare(a, s);
    }
    void cycle(size_t l, const T* b, T* x, hipStream_t s) {
        if (l + 1 == S.size()) {
            dense_mv<T>(ncoarse, cinv, b, x, s);
            return;
        }
        LS& q = S[l];
        const LevelSetup& ls = L[l];
        hgs<T, 1>(ls.A, q.av, q.dinv, q.ell, b, nullptr, q.w, false, s);
        sell_mv<T>(q.A, q.w, b, q.r, 1, s);
        bsrt_mv<T>(q.R, q.r, S[l + 1].b, s);
        cycle(l + 1, S[l + 1].b, S[l + 1].x, s);
        sell_mv<T>(q.P, S[l + 1].x, nullptr, q.w, 2, s);
        hgs<T, 1>(ls.A, q.av, q.dinv, q.ell, b, q.w, x, true, s);
    }
    void cycle3(size_t l, const T* b, T* x, hipStream_t s) {
        if (l + 1 == S.size()) {
            dense_mv3<T>(ncoarse, cinv, b, x, s);
            return;
        }
        LS& q = S[l];
        const LevelSetup& ls = L[l];
        hgs<T, 3>(ls.A, q.av, q.dinv, q.ell, b, nullptr, q.w3, false, s);
        sell_mv3<T>(q.A, q.w3, b, q.r3, 1, s);
        bsrt_mv3<T>(q.R, q.r3, S[l + 1].b3, s);
        cycle3(l + 1, S[l + 1].b3, S[l + 1].x3, s);
        sell_mv3<T>(q.P, S[l + 1].x3, nullptr, q.w3, 2, s);
        hgs<T, 3>(ls.A, q.av, q.dinv, q.ell, b, q.w3, x, true, s);
    }
    void vcycle(const double* x, double* y, hipStream_t s) override {
        ++vcycles;
        if constexpr (std::is_same<T, double>::value) {
            cycle(0, x, y, s);
        } else {
            const int64_t n = n0();
            cast_d2f(x, S[0].b, n, s);
            cycle(0, S[0].b, S[0].x, s);
            cast_f2d(S[0].x, y, n, s);
        }
    }
    void vcycle3(const double* x, double* y, hipStream_t s) override {
        if (!three) throw Error(SCR_E_INVALID, "three-column V-cycle on a hierarchy built without it");
        vcycles += 3;
        if constexpr (std::is_same<T, double>::value) {
            cycle3(0, x, y, s);
        } else {
            const int64_t n = n0();
            cast_d2f(x, S[0].b3, 3 * n, s);
            cycle3(0, S[0].b3, S[0].x3, s);
            cast_f2d(S[0].x3, y, 3 * n, s);
        }
    }
    void vcycle_f(const float* x, float* y, hipStream_t s) override {
        if constexpr (std::is_same<T, float>::value) {
            ++vcycles;
            cycle(0, x, y, s);
        } else {
            throw Error(SCR_E_INVALID, "FP32 V-cycle on an FP64 hierarchy");
        }
    }
    const DSell<float>* level0_f() const override {
        if constexpr (std::is_same<T, float>::value) {
            return S.size() < 2 ? nullptr : &S[0].A;
        } else {
            return nullptr;
        }
    }
};

int read_flag(const int* p, hipStream_t s) {
    int v = 0;
    HIPCHK(hipMemcpyAsync(&v, p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return v;
}

// transpose map of a structurally symmetric pattern (throws otherwise)
int32_t* transpose_map(int64_t nr, const int32_t* rp, const int32_t* ci, int64_t nnz, int* err, Arena& ar, hipStream_t s) {
    int32_t* tmap = ar.make<int32_t>(nnz + 1);
    zero_dev(err, sizeof(int), s);
    if (nr) tmap_k<<<(unsigned)cdiv(nr, 256), 256, 0, s>>>(nr, rp, ci, tmap, err);
    check_launch("transpose map");
    if (read_flag(err, s)) throw Error(SCR_E_INVALID, "classical AMG needs a structurally symmetric matrix");
    return tmap;
}

// HMIS C/F split of the graph (rp, ci, S) with its transpose map: returns the number of C points
// and their indices in *cidx (allocated; -1 on F points)
int64_t hmis(int64_t nr, const int32_t* rp, const int32_t* ci, const uint8_t* S, const int32_t* tmap, uint64_t seed,
             int level, int* err, Arena& ar, hipStream_t s, int32_t** cidx) {
    const unsigned g = (unsigned)cdiv(nr > 0 ? nr : 1, 256);
    int8_t* first = ar.make<int8_t>(nr + 1);
    double* w = ar.make<double>(nr + 1);
    int8_t* st = ar.make<int8_t>(nr + 1);
    int8_t* st2 = ar.make<int8_t>(nr + 1);
    uint8_t* isnew = ar.make<uint8_t>(nr + 1);
    if (nr) {
        hmis_first_k<<<(unsigned)cdiv(nr, HMIS_DOM), HMIS_DOM, 0, s>>>(nr, rp, ci, S, tmap, first);
        check_launch("hmis first pass");
        pmis_init_k<<<g, 256, 0, s>>>(nr, rp, ci, S, tmap, first, seed, level, w, st, isnew);
        check_launch("pmis init");
        for (int round = 0;; ++round) {
            if (round > 100000) throw Error(SCR_E_HIP, "PMIS did not terminate");
            zero_dev(err, sizeof(int), s);
            pmis_f_k<<<g, 256, 0, s>>>(nr, rp, ci, S, isnew, st, st2, err);
            check_launch("pmis f");
            std::swap(st, st2);
            if (read_flag(err, s) == 0) break;
            pmis_c_k<<<g, 256, 0, s>>>(nr, rp, ci, S, tmap, w, st, isnew);
            pmis_apply_k<<<g, 256, 0, s>>>(nr, isnew, st);
            check_launch("pmis c");
        }
    }
    int32_t* f = ar.make<int32_t>(nr + 1);
    int32_t* rank = ar.make<int32_t>(nr + 1);
    if (nr) cflag_k<<<g, 256, 0, s>>>(nr, st, f);
    const int64_t nc = scan_i32(f, rank, nr, ar, s);
    *cidx = ar.make<int32_t>(nr + 1);
    if (nr) cidx_k<<<g, 256, 0, s>>>(nr, st, rank, *cidx);
    check_launch("coarse index");
    ar.free(f); ar.free(rank); ar.free(first); ar.free(w); ar.free(st); ar.free(st2); ar.free(isnew);
    return nc;
}

// extended+i interpolation (nr x nc, 1x1) of (A, func, S) onto the C points of cidx
DBsr extpi(const DBsr& A, const uint8_t* func, const uint8_t* S, const int32_t* cidx, int64_t nc,
           const scr_amg_opts& o, Arena& ar, hipStream_t s) {
    const int64_t nr = A.nr;
    const unsigned g = (unsigned)cdiv(nr > 0 ? nr : 1, 256);
    int32_t* cap = ar.make<int32_t>(nr + 1);
    int32_t* off = ar.make<int32_t>(nr + 1);
    if (nr) extpi_cap_k<<<g, 256, 0, s>>>(nr, A.rp, A.ci, S, cidx, cap);
    check_launch("extpi cap");
    const int64_t total = scan_i32(cap, off, nr, ar, s);
    if (total >= INT32_MAX) throw Error(SCR_E_OOM, "interpolation candidates exceed 2^31");
    int32_t* hcol = ar.make<int32_t>(total + 1);
    double* hw = ar.make<double>(total + 1);
    int32_t* cnt = ar.make<int32_t>(nr + 1);
    if (nr) extpi_row_k<<<g, 256, 0, s>>>(nr, A.rp, A.ci, A.v, func, S, cidx, off, o.trunc, o.pmax, hcol, hw, cnt);
    check_launch("extpi rows");
    DBsr P;
    P.nr = nr; P.nc = nc; P.br = 1; P.bc = 1;
    P.rp = ar.make<int32_t>(nr + 1);
    P.nnzb = scan_i32(cnt, P.rp, nr, ar, s);
    P.ci = ar.make<int32_t>(P.nnzb + 1);
    P.v = ar.make<double>(P.nnzb + 1);
    if (nr) extpi_fill_k<<<g, 256, 0, s>>>(nr, off, hcol, hw, P.rp, P.ci, P.v);
    check_launch("extpi fill");
    ar.free(cap); ar.free(off); ar.free(hcol); ar.free(hw); ar.free(cnt);
    return P;
}

// the rows of P truncated as one interpolation row each, into a new matrix (P released)
DBsr truncate_matrix(DBsr& P, const scr_amg_opts& o, Arena& ar, hipStream_t s) {
    const int64_t nr = P.nr;
    const unsigned g = (unsigned)cdiv(nr > 0 ? nr : 1, 256);
    int32_t* cnt = ar.make<int32_t>(nr + 1);
    if (nr) trunc_rows_k<<<g, 256, 0, s>>>(nr, P.rp, P.ci, P.v, o.trunc, o.pmax, cnt);
    check_launch("truncate rows");
    DBsr T;
    T.nr = nr; T.nc = P.nc; T.br = 1; T.bc = 1;
    T.rp = ar.make<int32_t>(nr + 1);
    T.nnzb = scan_i32(cnt, T.rp, nr, ar, s);
    T.ci = ar.make<int32_t>(T.nnzb + 1);
    T.v = ar.make<double>(T.nnzb + 1);
    if (nr) extpi_fill_k<<<g, 256, 0, s>>>(nr, P.rp, P.ci, P.v, T.rp, T.ci, T.v);
    check_launch("truncate fill");
    ar.free(cnt);
    bsr_release(P, ar);
    return T;
}

// One standard level: HMIS on S and extended+i onto its C points (L.agg, L.P); returns the number
// of coarse points
int64_t standard_level(LevelSetup& L, const int32_t* tmap, const scr_amg_opts& o, int l, int* err, Arena& ar,
                       hipStream_t s) {
    const int64_t nc = hmis(L.A.nr, L.A.rp, L.A.ci, L.strong, tmap, o.seed, l, err, ar, s, &L.agg);
    if (nc > 0) L.P = extpi(L.A, L.func, L.strong, L.agg, nc, o, ar, s);
    return nc;
}

// One aggressive level: HMIS on S (first stage), HMIS on the second-stage graph of its C points,
// P = truncation of P1 P2 (P1: extended+i of A onto the first-stage C points; P2: extended+i of
// A1 = P1^T A P1 onto the kept ones)
int64_t aggressive_level(LevelSetup& L, const int32_t* tmap, const scr_amg_opts& o, int l, int* err, Arena& ar,
                         hipStream_t s) {
    const int64_t nr = L.A.nr;
    const unsigned g = (unsigned)cdiv(nr > 0 ? nr : 1, 256);
    int32_t* c1 = nullptr;
    const int64_t n1 = hmis(nr, L.A.rp, L.A.ci, L.strong, tmap, o.seed, l, err, ar, s, &c1);
    const unsigned g1 = (unsigned)cdiv(n1 > 0 ? n1 : 1, 256);
    // the second-stage graph (symmetric pattern, flags on the edges)
    int32_t* fine_of = ar.make<int32_t>(n1 + 1);
    int32_t* cap = ar.make<int32_t>(n1 + 1);
    int32_t* off = ar.make<int32_t>(n1 + 1);
    if (nr) fine_of_k<<<g, 256, 0, s>>>(nr, c1, fine_of);
    if (n1) ss_cap_k<<<g1, 256, 0, s>>>(n1, fine_of, L.A.rp, L.A.ci, L.strong, cap);
    check_launch("second stage cap");
    const int64_t tot = scan_i32(cap, off, n1, ar, s);
    if (tot >= INT32_MAX) throw Error(SCR_E_OOM, "second-stage candidates exceed 2^31");
    int32_t* buf = ar.make<int32_t>(tot + 1);
    int32_t* no = ar.make<int32_t>(n1 + 1);
    int32_t* nin = ar.make<int32_t>(n1 + 1);
    zero_dev(nin, (n1 + 1) * sizeof(int32_t), s);
    if (n1) {
        ss_out_k<<<g1, 256, 0, s>>>(n1, fine_of, L.A.rp, L.A.ci, L.strong, c1, off, buf, no);
        ss_indeg_k<<<g1, 256, 0, s>>>(n1, off, buf, no, nin);
    }
    check_launch("second stage out-edges");
    int32_t* inoff = ar.make<int32_t>(n1 + 1);
    const int64_t tin = scan_i32(nin, inoff, n1, ar, s);
    int32_t* inbuf = ar.make<int32_t>(tin + 1);
    int32_t* cur = ar.make<int32_t>(n1 + 1);
    zero_dev(cur, (n1 + 1) * sizeof(int32_t), s);
    int32_t* cnt = ar.make<int32_t>(n1 + 1);
    if (n1) {
        ss_in_fill_k<<<g1, 256, 0, s>>>(n1, off, buf, no, inoff, cur, inbuf);
        ss_in_sort_k<<<g1, 256, 0, s>>>(n1, inoff, nin, inbuf);
        ss_merge_k<false><<<g1, 256, 0, s>>>(n1, off, buf, no, inoff, inbuf, nin, nullptr, nullptr, nullptr, cnt);
    }
    check_launch("second stage in-edges");
    DBsr G;
    G.nr = G.nc = n1; G.br = G.bc = 1;
    G.rp = ar.make<int32_t>(n1 + 1);
    G.nnzb = scan_i32(cnt, G.rp, n1, ar, s);
    if (G.nnzb >= INT32_MAX) throw Error(SCR_E_OOM, "second-stage graph exceeds 2^31 entries");
    G.ci = ar.make<int32_t>(G.nnzb + 1);
    uint8_t* gS = ar.make<uint8_t>(G.nnzb + 1);
    if (n1) ss_merge_k<true><<<g1, 256, 0, s>>>(n1, off, buf, no, inoff, inbuf, nin, G.rp, G.ci, gS, nullptr);
    check_launch("second stage pattern");
    for (void* p : {(void*)cap, (void*)off, (void*)buf, (void*)no, (void*)nin, (void*)inoff, (void*)inbuf, (void*)cur,
                    (void*)cnt, (void*)fine_of})
        ar.free(p);
    int32_t* gmap = transpose_map(n1, G.rp, G.ci, G.nnzb, err, ar, s);
    int32_t* c2 = nullptr;
    const int64_t n2 = hmis(n1, G.rp, G.ci, gS, gmap, o.seed, l + 32, err, ar, s, &c2);
    ar.free(gmap); ar.free(gS); ar.free(G.rp); ar.free(G.ci);
    L.agg = ar.make<int32_t>(nr + 1);
    if (nr) agg_compose_k<<<g, 256, 0, s>>>(nr, c1, c2, L.agg);
    check_launch("aggressive coarse index");
    if (n2 > 0) {
        DBsr P1 = extpi(L.A, L.func, L.strong, c1, n1, o, ar, s);
        DBsr R1 = transpose(P1, ar, s);
        DBsr AP1 = spgemm(L.A, P1, nullptr, ar, s);
        DBsr A1 = spgemm(R1, AP1, nullptr, ar, s);
        bsr_release(R1, ar);
        bsr_release(AP1, ar);
        uint8_t* f1 = ar.make<uint8_t>(n1 + 1);
        if (nr) coarse_func_k<<<g, 256, 0, s>>>(nr, c1, L.func, f1);
        uint8_t* S1 = ar.make<uint8_t>(A1.nnzb + 1);
        if (n1) cl_strength_k<<<g1, 256, 0, s>>>(n1, A1.rp, A1.ci, A1.v, f1, o.cl_theta, S1);
        check_launch("first-stage coarse strength");
        DBsr P2 = extpi(A1, f1, S1, c2, n2, o, ar, s);
        DBsr P12 = spgemm(P1, P2, nullptr, ar, s);
        L.P = truncate_matrix(P12, o, ar, s);
        bsr_release(P1, ar);
        bsr_release(P2, ar);
        bsr_release(A1, ar);
        ar.free(f1);
        ar.free(S1);
    }
    ar.free(c1);
    ar.free(c2);
    return n2;
}

// every level of the classical hierarchy into H (H.L empty on entry; level 0 from A0)
void setup_levels(ClassicalBase& H, const DBsr& A0, const scr_amg_opts& o, Arena& ar, hipStream_t s) {
    int* err = ar.make<int>(1);
    unsigned long long* lamd = ar.make<unsigned long long>(1);
    {
        LevelSetup l0;
        const int b = A0.br;
        const int64_t n = A0.nr * b;
        l0.A = bsr_alloc(n, A0.nc * b, 1, 1, A0.nnzb * b * b, ar);
        l0.b = 1; l0.k = 1;
        l0.func = ar.make<uint8_t>(n > 0 ? n : 1);
        if (A0.nr) to_scalar_k<<<(unsigned)cdiv(A0.nr, 256), 256, 0, s>>>(A0.nr, b, A0.rp, A0.ci, A0.v, l0.A.rp, l0.A.ci,
                                                                          l0.A.v, l0.func);
        else zero_dev(l0.A.rp, sizeof(int32_t), s);
        check_launch("to_scalar");
        H.L.push_back(l0);
    }
    for (int l = 0;; ++l) {
        LevelSetup& L = H.L[l];
        const int64_t nr = L.A.nr;
        const unsigned g = (unsigned)cdiv(nr, 256);
        L.Dinv = ar.make<double>(nr > 0 ? nr : 1);
        level_diag(L, l, err, lamd, s);
        if (o.l1_gs) {
            L.ell = ar.make<double>(nr > 0 ? nr : 1);
            if (nr) l1_diag_k<<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.A.v, L.ell, L.Dinv);
            check_launch("l1 diagonal");
        }
        if (nr <= o.coarse_max || l + 1 >= o.max_levels || l + 1 >= 16) break;
        int32_t* tmap = transpose_map(nr, L.A.rp, L.A.ci, L.A.nnzb, err, ar, s);
        L.strong = ar.make<uint8_t>(L.A.nnzb + 1);
        cl_strength_k<<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.A.v, L.func, o.cl_theta, L.strong);
        check_launch("classical strength");
        const int64_t nc = l < o.agg_levels ? aggressive_level(L, tmap, o, l, err, ar, s)
                                            : standard_level(L, tmap, o, l, err, ar, s);
        ar.free(tmap);
        if (nc <= 0 || (double)nc > o.max_coarse_ratio * (double)nr) {
            ar.free(L.agg); L.agg = nullptr;
            ar.free(L.strong); L.strong = nullptr;
            bsr_release(L.P, ar);
            break;
        }
        L.nagg = nc;
        L.R = transpose(L.P, ar, s);
        DBsr AP = spgemm(L.A, L.P, nullptr, ar, s);
        LevelSetup N;
        N.A = spgemm(L.R, AP, nullptr, ar, s);
        bsr_release(AP, ar);
        N.b = 1; N.k = 1;
        N.func = ar.make<uint8_t>(nc);
        coarse_func_k<<<g, 256, 0, s>>>(nr, L.agg, L.func, N.func);
        check_launch("coarse functions");
        H.L.push_back(N);   // invalidates L
    }
    coarse_inverse(H, err, ar, s);
    ar.free(err);
    ar.free(lamd);
}

void release_levels(ClassicalBase& H, Arena& ar) {
    H.release_solve(ar);
    for (LevelSetup& L : H.L) {
        bsr_release(L.A, ar);
        bsr_release(L.P, ar);
        bsr_release(L.R, ar);
        for (void* p : {(void*)L.agg, (void*)L.strong, (void*)L.Dinv, (void*)L.func, (void*)L.ell}) ar.free(p);
    }
    H.L.clear();
    if (H.cinv) { ar.free(H.cinv); H.cinv = nullptr; }
}

}  // namespace

std::unique_ptr<Hierarchy> build_classical(const DBsr& A0, const scr_amg_opts& o, Arena& ar, hipStream_t s, bool three) {
    if (A0.br != A0.bc || A0.br < 1 || A0.br > 6) throw Error(SCR_E_INVALID, "classical AMG: square blocks up to 6x6");
    if (three && A0.br != 1) throw Error(SCR_E_INVALID, "three-column V-cycles need a scalar matrix");
    std::unique_ptr<ClassicalBase> H;
    if (o.precision == SCR_FP64) H.reset(new ClassicalHier<double>());
    else H.reset(new ClassicalHier<float>());
    H->opts = o;
    H->three = three;
    DBsr& p0 = H->pattern0;
    p0.nr = A0.nr; p0.nc = A0.nc; p0.br = A0.br; p0.bc = A0.bc; p0.nnzb = A0.nnzb;
    p0.rp = ar.make<int32_t>(A0.nr + 1);
    p0.ci = ar.make<int32_t>(A0.nnzb + 1);
    copy_dev(p0.rp, A0.rp, (A0.nr + 1) * sizeof(int32_t), s);
    copy_dev(p0.ci, A0.ci, A0.nnzb * sizeof(int32_t), s);
    setup_levels(*H, A0, o, ar, s);
    H->prepare(ar, s);
    HIPCHK(hipStreamSynchronize(s));
    return std::unique_ptr<Hierarchy>(H.release());
}

void update_classical(Hierarchy& Hb, const double* vals0, Arena& ar, hipStream_t s) {
    ClassicalBase& H = static_cast<ClassicalBase&>(Hb);
    // the splitting and the interpolation depend on the values: set the hierarchy up again on
    // the kept block pattern of level 0
    release_levels(H, ar);
    DBsr A0 = H.pattern0;
    A0.v = const_cast<double*>(vals0);
    setup_levels(H, A0, H.opts, ar, s);
    H.prepare(ar, s);
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace scr
