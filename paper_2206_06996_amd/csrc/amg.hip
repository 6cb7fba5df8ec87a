// amg.hip -- smoothed-aggregation AMG setup on the GPU and the V-cycle.
//
// Per level: strength graph (squared Frobenius block norms f_ij, strong iff
// f_ij^2 >= theta^4 f_ii f_jj, symmetrised by OR) -> distance-2 maximal independent set by
// synchronous rounds over seeded priorities (equal to the sequential greedy set in descending
// priority order) -> aggregates -> tentative prolongator by Gram-Schmidt of the near-null space
// on each aggregate -> P = (I - omega D^-1 A) P_tent, omega = 4/(3 lambda_hat) -> R = P^T ->
// A_c = R (A P), all products on structural patterns -> dense inverse of the coarsest level.
// The paper (Sec. 5.2) preconditions with BoomerAMG; smoothed aggregation replaces it here.
//
// Built with -ffp-contract=off: the strength predicate and the Gram-Schmidt decisions are
// evaluated as written, without fused multiply-adds.
#include <algorithm>
#include <cmath>

#include "solver.h"

namespace scr {

// ====================================================================== helpers
__device__ __forceinline__ int32_t find_col(const int32_t* __restrict__ ci, int32_t lo, int32_t hi, int32_t c) {
    int32_t e = hi;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (ci[mid] < c) lo = mid + 1; else hi = mid;
    }
    return (lo < e && ci[lo] == c) ? lo : -1;
}

// first index in [lo, hi) whose column is >= c (hi if none)
__device__ __forceinline__ int32_t lower_col(const int32_t* __restrict__ ci, int32_t lo, int32_t hi, int32_t c) {
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (ci[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}
// priority of node i at a level: 30 bits of splitmix64(seed, level, i) above the index
__device__ __forceinline__ uint64_t mis_key(uint64_t seed, int level, int64_t i) {
    uint64_t h = sm64(seed ^ ((uint64_t)level << 56) ^ ((uint64_t)i * 0xD1B54A32D192ED03ULL));
    return ((h >> 34) << 32) | (uint64_t)(uint32_t)i;
}

DBsr bsr_alloc(int64_t nr, int64_t nc, int br, int bc, int64_t nnzb, Arena& ar) {
    DBsr M;
    M.nr = nr; M.nc = nc; M.br = br; M.bc = bc; M.nnzb = nnzb;
    M.rp = ar.make<int32_t>(nr + 1);
    M.ci = ar.make<int32_t>(nnzb > 0 ? nnzb : 1);
    M.v = ar.make<double>((nnzb > 0 ? nnzb : 1) * br * bc);
    return M;
}
void bsr_release(DBsr& M, Arena& ar) {
    ar.free(M.rp); ar.free(M.ci); ar.free(M.v);
    M = DBsr();
}

// ====================================================================== block split and S^
__global__ void split_k(int64_t nnzb, const double* __restrict__ K, double* __restrict__ A, double* __restrict__ G,
                        double* __restrict__ D, double* __restrict__ C) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnzb) return;
    const double* k = K + q * 16;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) A[q * 9 + 3 * i + j] = k[4 * i + j];
        G[q * 3 + i] = k[4 * i + 3];
        D[q * 3 + i] = k[12 + i];
    }
    C[q] = k[15];
}

void split_values(const DBsr& K, DBsr& A, DBsr& G, DBsr& D, DBsr& C, hipStream_t s) {
    if (K.nnzb > 0) split_k<<<cdiv(K.nnzb, 256), 256, 0, s>>>(K.nnzb, K.v, A.v, G.v, D.v, C.v);
    check_launch("split");
}

void split_blocks(const DBsr& K, DBsr& A, DBsr& G, DBsr& D, DBsr& C, Arena& ar, hipStream_t s) {
    auto mk = [&](DBsr& M, int br, int bc) {
        M.nr = K.nr; M.nc = K.nc; M.br = br; M.bc = bc; M.nnzb = K.nnzb;
        M.rp = K.rp; M.ci = K.ci;          // index arrays shared with K
        M.v = ar.make<double>(K.nnzb * br * bc);
    };
    mk(A, 3, 3); mk(G, 3, 1); mk(D, 1, 3); mk(C, 1, 1);
    if (K.nnzb > 0) split_k<<<cdiv(K.nnzb, 256), 256, 0, s>>>(K.nnzb, K.v, A.v, G.v, D.v, C.v);
    check_launch("split");
}

// ====================================================================== generic SpGEMM (one wave per row)
constexpr int HS_MAX = 8192;       // largest LDS hash table per row
constexpr int HMAX = HS_MAX / 2;   // unique columns allowed per row
constexpr int HS_COUNT = 2048;     // first hash table of the counting pass (x4 on each overflow)
constexpr int SPG_NW_BOUND = 2048; // mean candidates per row from which rows take four wavefronts

// returns 1 if newly inserted (table of hs slots, hs a power of two, never more than half full)
__device__ __forceinline__ int hash_insert(int* t, int hs, int key) {
    unsigned h = ((unsigned)key * 2654435761u) & (unsigned)(hs - 1);
    for (;;) {
        int prev = atomicCAS(&t[h], -1, key);
        if (prev == -1) return 1;
        if (prev == key) return 0;
        h = (h + 1) & (unsigned)(hs - 1);
    }
}

// Maximum over a 256-thread workgroup, folded into *out by one atomic (every thread must call it).
// A same-address atomic per row serialises at one L2 channel: 324k of them cost about 3.5 ms.
template <typename T>
__device__ __forceinline__ void block_max_to(T v, T* out) {
    __shared__ T red[256 / WAVE];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, WAVE);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T m = red[0];
        for (int w = 1; w < 256 / WAVE; ++w) m = red[w] > m ? red[w] : m;
        atomicMax(out, m);
    }
}

// upper bound of the candidates of each row of X*Y (sum of the lengths of the Y rows it meets):
// its maximum over the rows into *maxub, its sum into *sumub.  A wavefront per row (grid-stride over
// the rows, at most SPG_BOUND_BLOCKS workgroups), one atomic of each kind per workgroup.
constexpr int SPG_BOUND_BLOCKS = 4096;
__global__ void __launch_bounds__(256) spg_bound_k(int64_t nr, const int32_t* __restrict__ xrp,
                                                   const int32_t* __restrict__ xci, const int32_t* __restrict__ yrp,
                                                   int* __restrict__ maxub, unsigned long long* __restrict__ sumub) {
    __shared__ int64_t redm[256 / WAVE];
    __shared__ unsigned long long reds[256 / WAVE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    int64_t mx = 0;
    unsigned long long sm = 0;
    for (int64_t i = (int64_t)blockIdx.x * (256 / WAVE) + w; i < nr; i += (int64_t)gridDim.x * (256 / WAVE)) {
        int64_t ub = 0;
        for (int32_t q = xrp[i] + lane; q < xrp[i + 1]; q += WAVE) {
            const int32_t k = xci[q];
            ub += yrp[k + 1] - yrp[k];
        }
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) ub += __shfl_xor(ub, o, WAVE);
        mx = ub > mx ? ub : mx;
        sm += (unsigned long long)ub;
    }
    if (lane == 0) { redm[w] = mx; reds[w] = sm; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 256 / WAVE; ++v) { mx = redm[v] > mx ? redm[v] : mx; sm += reds[v]; }
        atomicMax(maxub, (int)(mx < (1 << 30) ? mx : (1 << 30)));
        atomicAdd(sumub, sm);
    }
}

// largest of n counts (one atomic per workgroup)
__global__ void __launch_bounds__(256) max_i32_k(int64_t n, const int32_t* __restrict__ a, int* __restrict__ out) {
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = a[i] > m ? a[i] : m;
    block_max_to(m, out);
}

// count (phase 0) or emit sorted (phase 1) the structural pattern of row i of X*Y, NW wavefronts
// per row sharing one LDS hash table (NW = 4 for products whose rows meet thousands of candidates:
// the table's LDS then serves four wavefronts instead of one).  In the counting pass a row whose
// unique columns overflow the table gets cnt = -1 and raises the overflow flag; a retry pass
// (retry = 1, larger table) recounts only those rows.
// Dynamic LDS: hs hash slots, then hs/2 + NW * 64 list entries.
template <int PHASE, int NW>
__global__ void __launch_bounds__(NW * WAVE) spg_symbolic(int64_t nr, int hs, int retry, const int32_t* __restrict__ xrp,
                                                          const int32_t* __restrict__ xci, const int32_t* __restrict__ yrp,
                                                          const int32_t* __restrict__ yci, const uint8_t* __restrict__ rowmask,
                                                          int32_t* __restrict__ cnt, const int32_t* __restrict__ crp,
                                                          int32_t* __restrict__ cci, int* __restrict__ overflow) {
    extern __shared__ int smem[];
    int* table = smem;
    int* list = smem + hs;
    __shared__ int nuniq;
    const int hmax = hs / 2;
    int64_t i = blockIdx.x;
    if (i >= nr) return;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    if (PHASE == 0 && retry && cnt[i] >= 0) return;
    if (rowmask && !rowmask[i]) {
        if (PHASE == 0 && tid == 0) cnt[i] = 0;
        return;
    }
    for (int t = tid; t < hs; t += NW * WAVE) table[t] = -1;
    if (tid == 0) nuniq = 0;
    __syncthreads();
    // The candidates (X entry q, Y entry t) of up to 64 X entries at a time are spread over the
    // lanes of one wavefront (wavefront w takes chunks w, w + NW, ...): lane l holds the Y row of
    // X entry q0 + l, an inclusive prefix of their lengths maps a candidate number to its (l, t) by
    // a binary search over the prefix (every lane takes part in the shuffles).  Only a set is
    // built here, so the order of insertion does not matter.
    const int32_t x0 = xrp[i], x1 = xrp[i + 1];
    for (int32_t q0 = x0 + (tid / WAVE) * WAVE; q0 < x1; q0 += NW * WAVE) {
        int st = 0, len = 0;
        if (q0 + lane < x1) {
            int32_t k = xci[q0 + lane];
            st = yrp[k];
            len = yrp[k + 1] - st;
        }
        int incl = len;
        for (int o = 1; o < WAVE; o <<= 1) {
            int v = __shfl_up(incl, o, WAVE);
            if (lane >= o) incl += v;
        }
        const int total = __shfl(incl, WAVE - 1, WAVE);
        for (int base = 0; base < total; base += WAVE) {
            if (nuniq >= hmax) break;
            const int cidx = base + lane;
            int l = 0;     // number of lanes whose inclusive prefix is <= cidx
            for (int step = WAVE / 2; step > 0; step >>= 1) {
                int v = __shfl(incl, l + step - 1, WAVE);
                if (v <= cidx) l += step;
            }
            const int stl = __shfl(st, l, WAVE);
            const int excl = __shfl(incl, l, WAVE) - __shfl(len, l, WAVE);
            if (cidx < total) {
                int c = yci[stl + (cidx - excl)];
                if (hash_insert(table, hs, c)) {
                    int pos = atomicAdd(&nuniq, 1);
                    if (pos < hmax + NW * WAVE) list[pos] = c;
                }
            }
        }
    }
    __syncthreads();
    int w = nuniq;
    if (w >= hmax) {
        if (tid == 0) {
            if (PHASE == 0) cnt[i] = -1;
            atomicOr(overflow, 1);
        }
        return;
    }
    if (PHASE == 0) {
        if (tid == 0) cnt[i] = w;
        return;
    }
    // rank sort of the unique columns
    int32_t base = crp[i];
    for (int a = tid; a < w; a += NW * WAVE) {
        int key = list[a], rank = 0;
        for (int b = 0; b < w; ++b) rank += list[b] < key;
        cci[base + rank] = key;
    }
}

// numeric phase: lane owns output blocks; accumulates X_iq * Y_kc over q in ascending order
template <int M, int N, int P>
__global__ void __launch_bounds__(256) spg_numeric(int64_t nr, const int32_t* __restrict__ xrp, const int32_t* __restrict__ xci,
                                                   const double* __restrict__ xv, const int32_t* __restrict__ yrp,
                                                   const int32_t* __restrict__ yci, const double* __restrict__ yv,
                                                   const int32_t* __restrict__ crp, const int32_t* __restrict__ cci,
                                                   double* __restrict__ cv) {
    int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (i >= nr) return;
    int lane = threadIdx.x & (WAVE - 1);
    for (int32_t p = crp[i] + lane; p < crp[i + 1]; p += WAVE) {
        int32_t c = cci[p];
        double acc[M * P];
        for (int e = 0; e < M * P; ++e) acc[e] = 0.0;
        for (int32_t q = xrp[i]; q < xrp[i + 1]; ++q) {
            int32_t k = xci[q];
            int32_t t = find_col(yci, yrp[k], yrp[k + 1], c);
            if (t < 0) continue;
            const double* xb = xv + (int64_t)q * M * N;
            const double* yb = yv + (int64_t)t * N * P;
            for (int r = 0; r < M; ++r)
                for (int cc = 0; cc < P; ++cc) {
                    double sum = 0.0;
                    for (int l = 0; l < N; ++l) sum += xb[r * N + l] * yb[l * P + cc];
                    acc[r * P + cc] += sum;
                }
        }
        double* o = cv + (int64_t)p * M * P;
        for (int e = 0; e < M * P; ++e) o[e] = acc[e];
    }
}

// numeric phase, one wave per output row: the row's output columns go into an LDS hash (column ->
// position).  The candidates (X entry q, Y entry t) of up to 64 X entries at a time are spread over
// all lanes as in the symbolic phase, each lane forms its block product X_iq * Y_kt in registers,
// and the products are added to their LDS accumulators in rounds: in each round the lowest pending
// lane of every accumulator (an LDS atomic minimum over lane ids) adds its product.  Lanes hold
// candidates in (q, t) order and a row of Y holds a column once, so every accumulator receives the
// same terms in the same order (q ascending) as in the pull kernel above and the results are
// identical; a round count is the largest number of candidates of one pass that meet one output
// column, instead of one serial step per X entry.  Where the rows of Y of a chunk of 64 X entries
// average SPG_STEP_LEN entries or more, the chunk instead takes one X entry per step with its row
// of Y over the lanes (the same order again), which costs less than packing rows that already fill
// the wave.
// Dynamic LDS: hs keys, hs positions, wmax * M * P doubles, then wmax owner slots.
constexpr int SPG_STEP_LEN = 32;
constexpr int SPG_PF = 4;
template <int M, int N, int P>
__global__ void __launch_bounds__(WAVE) spg_numeric_lds(int64_t nr, int hs, int wmax, const int32_t* __restrict__ xrp,
                                                        const int32_t* __restrict__ xci, const double* __restrict__ xv,
                                                        const int32_t* __restrict__ yrp, const int32_t* __restrict__ yci,
                                                        const double* __restrict__ yv, const int32_t* __restrict__ crp,
                                                        const int32_t* __restrict__ cci, double* __restrict__ cv) {
    extern __shared__ int smem[];
    int* keys = smem;
    int* pos = smem + hs;
    double* acc = reinterpret_cast<double*>(smem + 2 * hs);
    constexpr int MP = M * P;
    int* owner = reinterpret_cast<int*>(acc + (size_t)wmax * MP);
    int64_t i = blockIdx.x;
    if (i >= nr) return;
    int lane = threadIdx.x;
    int32_t c0 = crp[i];
    int w = crp[i + 1] - c0;
    if (w == 0) return;
    for (int t = lane; t < hs; t += WAVE) keys[t] = -1;
    __syncthreads();
    for (int p = lane; p < w; p += WAVE) {
        int c = cci[c0 + p];
        unsigned h = ((unsigned)c * 2654435761u) & (unsigned)(hs - 1);
        while (atomicCAS(&keys[h], -1, c) != -1) h = (h + 1) & (unsigned)(hs - 1);
        pos[h] = p;
        owner[p] = WAVE;
        for (int e = 0; e < MP; ++e) acc[p * MP + e] = 0.0;
    }
    __syncthreads();
    const int32_t x0 = xrp[i], x1 = xrp[i + 1];
    for (int32_t q0 = x0; q0 < x1; q0 += WAVE) {
        int st = 0, len = 0;
        if (q0 + lane < x1) {
            int32_t k = xci[q0 + lane];
            st = yrp[k];
            len = yrp[k + 1] - st;
        }
        int incl = len;
        for (int o = 1; o < WAVE; o <<= 1) {
            int v = __shfl_up(incl, o, WAVE);
            if (lane >= o) incl += v;
        }
        const int total = __shfl(incl, WAVE - 1, WAVE);
        const int nq = x1 - q0 < WAVE ? x1 - q0 : WAVE;
        if (total >= SPG_STEP_LEN * nq) {
            // long rows of Y: one X entry per step, its row of Y over the lanes
            if constexpr (M == 1 && N == 1 && P == 1) {
                // scalar: the first 64 entries of the Y rows of SPG_PF steps are loaded together
                // before those steps run in order (the same terms, order and arithmetic as below)
                const double xl = lane < nq ? xv[q0 + lane] : 0.0;
                for (int j0 = 0; j0 < nq; j0 += SPG_PF) {
                    int cpf[SPG_PF];
                    double ypf[SPG_PF];
#pragma unroll
                    for (int u = 0; u < SPG_PF; ++u) {
                        cpf[u] = -1;
                        ypf[u] = 0.0;
                        if (j0 + u < nq) {
                            const int stj = __builtin_amdgcn_readlane(st, j0 + u);
                            if (lane < __builtin_amdgcn_readlane(len, j0 + u)) {
                                cpf[u] = yci[stj + lane];
                                ypf[u] = yv[stj + lane];
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < SPG_PF; ++u) {
                        const int j = j0 + u;
                        if (j >= nq) break;
                        const double xj = __shfl(xl, j, WAVE);
                        const int stj = __builtin_amdgcn_readlane(st, j);
                        const int enj = stj + __builtin_amdgcn_readlane(len, j);
                        for (int32_t t = stj + lane; t < enj; t += WAVE) {
                            const int c = t == stj + lane ? cpf[u] : yci[t];
                            const double y = t == stj + lane ? ypf[u] : yv[t];
                            unsigned h = ((unsigned)c * 2654435761u) & (unsigned)(hs - 1);
                            for (int g = 0; g < hs && keys[h] != c; ++g) h = (h + 1) & (unsigned)(hs - 1);
                            if (keys[h] != c) continue;   // not reached: every column met is in the pattern
                            double sum = 0.0;
                            sum += xj * y;
                            acc[pos[h]] += sum;
                        }
                        __syncthreads();
                    }
                }
                continue;
            }
            for (int j = 0; j < nq; ++j) {
                const int stj = __builtin_amdgcn_readlane(st, j);
                const int enj = stj + __builtin_amdgcn_readlane(len, j);
                const double* xb = xv + (int64_t)(q0 + j) * M * N;
                for (int t = stj + lane; t < enj; t += WAVE) {
                    const int c = yci[t];
                    unsigned h = ((unsigned)c * 2654435761u) & (unsigned)(hs - 1);
                    for (int g = 0; g < hs && keys[h] != c; ++g) h = (h + 1) & (unsigned)(hs - 1);
                    if (keys[h] != c) continue;       // not reached: every column met is in the pattern
                    double* a = acc + pos[h] * MP;
                    const double* yb = yv + (int64_t)t * N * P;
                    for (int r = 0; r < M; ++r)
                        for (int cc = 0; cc < P; ++cc) {
                            double sum = 0.0;
                            for (int k = 0; k < N; ++k) sum += xb[r * N + k] * yb[k * P + cc];
                            a[r * P + cc] += sum;
                        }
                }
                __syncthreads();
            }
            continue;
        }
        for (int base = 0; base < total; base += WAVE) {
            const int cidx = base + lane;
            int l = 0;     // number of lanes whose inclusive prefix is <= cidx
            for (int step = WAVE / 2; step > 0; step >>= 1) {
                int v = __shfl(incl, l + step - 1, WAVE);
                if (v <= cidx) l += step;
            }
            const int stl = __shfl(st, l, WAVE);
            const int excl = __shfl(incl, l, WAVE) - __shfl(len, l, WAVE);
            bool todo = false;
            int p = 0;
            double prod[MP];
            if (cidx < total) {
                const int32_t t = stl + (cidx - excl);
                const int c = yci[t];
                unsigned h = ((unsigned)c * 2654435761u) & (unsigned)(hs - 1);
                for (int g = 0; g < hs && keys[h] != c; ++g) h = (h + 1) & (unsigned)(hs - 1);
                todo = keys[h] == c;       // always: every column met is in the pattern
                p = pos[h];
                const double* xb = xv + (int64_t)(q0 + l) * M * N;
                const double* yb = yv + (int64_t)t * N * P;
                for (int r = 0; r < M; ++r)
                    for (int cc = 0; cc < P; ++cc) {
                        double sum = 0.0;
                        for (int k = 0; k < N; ++k) sum += xb[r * N + k] * yb[k * P + cc];
                        prod[r * P + cc] = sum;
                    }
            }
            while (__ballot(todo)) {
                if (todo) atomicMin(&owner[p], lane);
                __syncthreads();
                if (todo && owner[p] == lane) {
                    for (int e = 0; e < MP; ++e) acc[p * MP + e] += prod[e];
                    owner[p] = WAVE;
                    todo = false;
                }
                __syncthreads();
            }
        }
    }
    for (int p = lane; p < w; p += WAVE)
        for (int e = 0; e < MP; ++e) cv[(int64_t)(c0 + p) * MP + e] = acc[p * MP + e];
}

// numeric phase of C = X Y into C's pattern (wmax = longest row of C): the LDS form when its
// accumulators fit, else the pull form
static void spgemm_numeric_run(const DBsr& X, const DBsr& Y, DBsr& C, int wmax, hipStream_t s) {
    int64_t nb = cdiv(X.nr, 4);
    int key = X.br * 100 + X.bc * 10 + Y.bc;
    int hsn = 64;
    while (hsn < 2 * wmax) hsn <<= 1;
    size_t lds_n = (size_t)2 * hsn * sizeof(int) + (size_t)wmax * (C.br * C.bc * sizeof(double) + sizeof(int));
    if (X.nr > 0 && lds_n <= 64 * 1024) {
#define SPL(m, n, p)                                                                                          \
    spg_numeric_lds<m, n, p><<<X.nr, WAVE, lds_n, s>>>(X.nr, hsn, wmax, X.rp, X.ci, X.v, Y.rp, Y.ci, Y.v, C.rp, C.ci, \
                                                       C.v)
        switch (key) {
            case 111: SPL(1, 1, 1); break;
            case 131: SPL(1, 3, 1); break;
            case 336: SPL(3, 3, 6); break;
            case 636: SPL(6, 3, 6); break;
            case 666: SPL(6, 6, 6); break;
            default: throw Error(SCR_E_UNIMPLEMENTED, "spgemm block shape " + std::to_string(key));
        }
#undef SPL
        check_launch("spg_numeric");
        return;
    }
#define SPN(m, n, p) spg_numeric<m, n, p><<<nb, 256, 0, s>>>(X.nr, X.rp, X.ci, X.v, Y.rp, Y.ci, Y.v, C.rp, C.ci, C.v)
    if (nb > 0) {
        switch (key) {
            case 111: SPN(1, 1, 1); break;
            case 131: SPN(1, 3, 1); break;
            case 336: SPN(3, 3, 6); break;
            case 636: SPN(6, 3, 6); break;
            case 666: SPN(6, 6, 6); break;
            default: throw Error(SCR_E_UNIMPLEMENTED, "spgemm block shape " + std::to_string(key));
        }
    }
#undef SPN
    check_launch("spg_numeric");
}

DBsr spgemm(const DBsr& X, const DBsr& Y, const uint8_t* rowmask, Arena& ar, hipStream_t s) {
    DBsr C;
    C.nr = X.nr; C.nc = Y.nc; C.br = X.br; C.bc = Y.bc;
    C.rp = ar.make<int32_t>(X.nr + 1);
    int32_t* cnt = ar.make<int32_t>(X.nr + 1);
    int* flags = ar.make<int>(3);      // [overflow, max candidate bound, max output row length]
    unsigned long long* csum = ar.make<unsigned long long>(1);   // candidates over all rows
    zero_dev(flags, 3 * sizeof(int), s);
    zero_dev(csum, sizeof(unsigned long long), s);
    if (X.nr > 0)
        spg_bound_k<<<(unsigned)std::min<int64_t>(cdiv(X.nr, 256 / WAVE), SPG_BOUND_BLOCKS), 256, 0, s>>>(
            X.nr, X.rp, X.ci, Y.rp, flags + 1, csum);
    int hflags[2] = {0, 0};
    unsigned long long hsum = 0;
    HIPCHK(hipMemcpyAsync(hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hsum, csum, sizeof(hsum), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(csum);
    // hash table of the counting pass: twice the candidate bound, but at most HS_COUNT slots (the
    // unique columns of a row are far fewer than its candidates); the rows that overflow it are
    // counted again with a table four times larger.  The result does not depend on the table size.
    // Products whose rows meet SPG_NW_BOUND candidates or more on average take four wavefronts
    // per row.
    const bool wide = X.nr > 0 && hsum >= (unsigned long long)SPG_NW_BOUND * (unsigned long long)X.nr;
    int need = 2 * (hflags[1] < HMAX ? hflags[1] : HMAX) + 2;
    int hs = 64;
    while (hs < need && hs < HS_COUNT) hs <<= 1;
    int hf[3] = {0, 0, 0};
    for (int retry = 0;; retry = 1) {
        if (X.nr > 0) {
            if (wide)
                spg_symbolic<0, 4><<<X.nr, 4 * WAVE, (size_t)(hs + hs / 2 + 4 * WAVE) * sizeof(int), s>>>(
                    X.nr, hs, retry, X.rp, X.ci, Y.rp, Y.ci, rowmask, cnt, nullptr, nullptr, flags);
            else
                spg_symbolic<0, 1><<<X.nr, WAVE, (size_t)(hs + hs / 2 + WAVE) * sizeof(int), s>>>(
                    X.nr, hs, retry, X.rp, X.ci, Y.rp, Y.ci, rowmask, cnt, nullptr, nullptr, flags);
        }
        check_launch("spg_count");
        HIPCHK(hipMemcpyAsync(hf, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!hf[0]) break;
        if (hs >= HS_MAX) throw Error(SCR_E_INVALID, "Galerkin product row wider than " + std::to_string(HMAX) + " blocks");
        hs = std::min(4 * hs, HS_MAX);
        zero_dev(flags, sizeof(int), s);
    }
    // widest output row (flags[2] is still zero: the counting pass does not touch it)
    if (X.nr > 0) max_i32_k<<<(unsigned)std::min<int64_t>(cdiv(X.nr, 256), 1024), 256, 0, s>>>(X.nr, cnt, flags + 2);
    check_launch("max_i32");
    HIPCHK(hipMemcpyAsync(&hf[2], flags + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    C.nnzb = scan_i32(cnt, C.rp, X.nr, ar, s);
    HIPCHK(hipStreamSynchronize(s));
    const int wmax = hf[2];
    ar.free(cnt);
    C.ci = ar.make<int32_t>(C.nnzb > 0 ? C.nnzb : 1);
    C.v = ar.make<double>((C.nnzb > 0 ? C.nnzb : 1) * C.br * C.bc);
    // the filling pass knows the widest row exactly
    int hs1 = 64;
    while (hs1 < 2 * wmax + 2) hs1 <<= 1;
    if (X.nr > 0) {
        if (wide)
            spg_symbolic<1, 4><<<X.nr, 4 * WAVE, (size_t)(hs1 + hs1 / 2 + 4 * WAVE) * sizeof(int), s>>>(
                X.nr, hs1, 0, X.rp, X.ci, Y.rp, Y.ci, rowmask, nullptr, C.rp, C.ci, flags);
        else
            spg_symbolic<1, 1><<<X.nr, WAVE, (size_t)(hs1 + hs1 / 2 + WAVE) * sizeof(int), s>>>(
                X.nr, hs1, 0, X.rp, X.ci, Y.rp, Y.ci, rowmask, nullptr, C.rp, C.ci, flags);
    }
    check_launch("spg_fill");
    ar.free(flags);
    spgemm_numeric_run(X, Y, C, wmax, s);
    return C;
}

// max row length of a pattern
__global__ void __launch_bounds__(256) rowlen_max_k(int64_t nr, const int32_t* __restrict__ rp, int* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    block_max_to(i < nr ? rp[i + 1] - rp[i] : 0, out);
}

// numeric phase only, into the existing pattern of C (same terms and order as a full product)
static void spgemm_numeric(const DBsr& X, const DBsr& Y, DBsr& C, Arena& ar, hipStream_t s) {
    int* d = ar.make<int>(1);
    zero_dev(d, sizeof(int), s);
    if (C.nr > 0) rowlen_max_k<<<cdiv(C.nr, 256), 256, 0, s>>>(C.nr, C.rp, d);
    int wmax = 0;
    HIPCHK(hipMemcpyAsync(&wmax, d, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(d);
    spgemm_numeric_run(X, Y, C, wmax, s);
}

// ---------------------------------------------------------------------- S^ = C - D d^-1 G
// d per velocity dof: the diagonal of A (mode 0) or the sum of the absolute values of its row
// (mode 1, SIMPLEC), summed block by block in column order
__global__ void schur_diag_k(int64_t nr, int mode, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const double* __restrict__ Av, double* __restrict__ d) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    if (mode == 0) {
        int32_t dq = find_col(ci, rp[i], rp[i + 1], (int32_t)i);
        for (int c = 0; c < 3; ++c) d[3 * i + c] = Av[(int64_t)dq * 9 + 4 * c];
        return;
    }
    for (int c = 0; c < 3; ++c) {
        double sum = 0.0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
            for (int k = 0; k < 3; ++k) sum += fabs(Av[(int64_t)q * 9 + 3 * c + k]);
        d[3 * i + c] = sum;
    }
}
__global__ void diag_scale_D(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const double* __restrict__ d, const double* __restrict__ Dv, double* __restrict__ X) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        int32_t j = ci[q];
        for (int c = 0; c < 3; ++c) X[(int64_t)q * 3 + c] = Dv[(int64_t)q * 3 + c] / d[3 * (int64_t)j + c];
    }
}
// union pattern of C and DG (both sorted, a column at most once per row): count, then fill with
// C - DG.  One wavefront per row: an entry's place in the union is its index in its own row, plus
// the entries of the other row with smaller columns, minus the columns the two rows share below it
// (a prefix count of the shared flags over its own row); a column in both rows is written once, by
// its C entry.
template <int PHASE>
__global__ void __launch_bounds__(256) merge_sub_k(int64_t nr, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                                   const double* __restrict__ av, const int32_t* __restrict__ brp,
                                                   const int32_t* __restrict__ bci, const double* __restrict__ bv,
                                                   int32_t* __restrict__ cnt, const int32_t* __restrict__ crp,
                                                   int32_t* __restrict__ cci, double* __restrict__ cv) {
    const int64_t i = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    if (i >= nr) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const uint64_t below = (1ull << lane) - 1;
    const int32_t a0 = arp[i], a1 = arp[i + 1], b0 = brp[i], b1 = brp[i + 1];
    const int32_t o = PHASE ? crp[i] : 0;
    int shared = 0;
    for (int32_t base = a0; base < a1; base += WAVE) {
        const int32_t a = base + lane;
        const bool in = a < a1;
        const int32_t ca = in ? aci[a] : 0;
        const int32_t lb = in ? lower_col(bci, b0, b1, ca) : b1;
        const bool m = in && lb < b1 && bci[lb] == ca;
        const uint64_t mask = __ballot(m);
        if (PHASE && in) {
            const int32_t pos = (a - a0) + (lb - b0) - (shared + __popcll(mask & below));
            cci[o + pos] = ca;
            cv[o + pos] = m ? av[a] - bv[lb] : av[a];
        }
        shared += __popcll(mask);
    }
    if (!PHASE) {
        if (lane == 0) cnt[i] = (a1 - a0) + (b1 - b0) - shared;
        return;
    }
    shared = 0;
    for (int32_t base = b0; base < b1; base += WAVE) {
        const int32_t b = base + lane;
        const bool in = b < b1;
        const int32_t cb = in ? bci[b] : 0;
        const int32_t la = in ? lower_col(aci, a0, a1, cb) : a1;
        const bool m = in && la < a1 && aci[la] == cb;
        const uint64_t mask = __ballot(m);
        if (in && !m) {
            const int32_t pos = (la - a0) + (b - b0) - (shared + __popcll(mask & below));
            cci[o + pos] = cb;
            cv[o + pos] = -bv[b];
        }
        shared += __popcll(mask);
    }
}

DBsr schur_approx(const DBsr& A, const DBsr& G, const DBsr& D, const DBsr& C, int mode, double* d, Arena& ar,
                  hipStream_t s) {
    DBsr X = D;
    X.v = ar.make<double>(D.nnzb * 3);
    if (A.nr > 0) schur_diag_k<<<cdiv(A.nr, 256), 256, 0, s>>>(A.nr, mode, A.rp, A.ci, A.v, d);
    if (D.nr > 0) diag_scale_D<<<cdiv(D.nr, 256), 256, 0, s>>>(D.nr, D.rp, D.ci, d, D.v, X.v);
    check_launch("diag_scale_D");
    DBsr DG = spgemm(X, G, nullptr, ar, s);
    ar.free(X.v);
    DBsr S;
    S.nr = C.nr; S.nc = C.nc; S.br = 1; S.bc = 1;
    S.rp = ar.make<int32_t>(C.nr + 1);
    int32_t* cnt = ar.make<int32_t>(C.nr + 1);
    int64_t nw = cdiv(C.nr, 256 / WAVE);
    if (nw) merge_sub_k<0><<<nw, 256, 0, s>>>(C.nr, C.rp, C.ci, C.v, DG.rp, DG.ci, DG.v, cnt, nullptr, nullptr, nullptr);
    S.nnzb = scan_i32(cnt, S.rp, C.nr, ar, s);
    ar.free(cnt);
    S.ci = ar.make<int32_t>(S.nnzb);
    S.v = ar.make<double>(S.nnzb);
    if (nw) merge_sub_k<1><<<nw, 256, 0, s>>>(C.nr, C.rp, C.ci, C.v, DG.rp, DG.ci, DG.v, nullptr, S.rp, S.ci, S.v);
    check_launch("merge_sub");
    bsr_release(DG, ar);
    return S;
}

void schur_update(const DBsr& A, const DBsr& G, const DBsr& D, const DBsr& C, int mode, double* d, DBsr& S, Arena& ar,
                  hipStream_t s) {
    DBsr X = D;
    X.v = ar.make<double>(D.nnzb * 3);
    if (A.nr > 0) schur_diag_k<<<cdiv(A.nr, 256), 256, 0, s>>>(A.nr, mode, A.rp, A.ci, A.v, d);
    if (D.nr > 0) diag_scale_D<<<cdiv(D.nr, 256), 256, 0, s>>>(D.nr, D.rp, D.ci, d, D.v, X.v);
    check_launch("diag_scale_D");
    DBsr DG = spgemm(X, G, nullptr, ar, s);
    ar.free(X.v);
    int64_t nw = cdiv(C.nr, 256 / WAVE);
    if (nw) merge_sub_k<1><<<nw, 256, 0, s>>>(C.nr, C.rp, C.ci, C.v, DG.rp, DG.ci, DG.v, nullptr, S.rp, S.ci, S.v);
    check_launch("merge_sub");
    bsr_release(DG, ar);
}

// ---------------------------------------------------------------------- rigid-body modes
__global__ void centroid_partial(int64_t nb, const double* __restrict__ xyz, double* __restrict__ part) {
    __shared__ double red[3][256];
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nb; i += (int64_t)gridDim.x * 256)
        for (int d = 0; d < 3; ++d) a[d] += xyz[3 * i + d];
    for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = a[d];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) part[blockIdx.x * 3 + d] = red[d][0];
}
__global__ void rigid_k(int64_t nb, const double* __restrict__ xyz, const double* __restrict__ part, int np,
                        double* __restrict__ B) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double c[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < np; ++p)
        for (int d = 0; d < 3; ++d) c[d] += part[p * 3 + d];
    double x = xyz[3 * i] - c[0] / (double)nb, y = xyz[3 * i + 1] - c[1] / (double)nb, z = xyz[3 * i + 2] - c[2] / (double)nb;
    double* r0 = B + (3 * i) * 6;
    double* r1 = r0 + 6;
    double* r2 = r1 + 6;
    for (int t = 0; t < 6; ++t) { r0[t] = 0.0; r1[t] = 0.0; r2[t] = 0.0; }
    r0[0] = 1.0; r1[1] = 1.0; r2[2] = 1.0;
    r0[3] = -y; r1[3] = x;
    r1[4] = -z; r2[4] = y;
    r0[5] = z; r2[5] = -x;
}
void rigid_modes(int64_t nb, const double* xyz, double* B, Arena& ar, hipStream_t s) {
    int np = 64;
    double* part = ar.make<double>(np * 3);
    centroid_partial<<<np, 256, 0, s>>>(nb, xyz, part);
    if (nb > 0) rigid_k<<<cdiv(nb, 256), 256, 0, s>>>(nb, xyz, part, np, B);
    check_launch("rigid_modes");
    ar.free(part);
}

// ====================================================================== strength and MIS-2
__device__ __forceinline__ double block_f(const double* __restrict__ v, int bb) {
    double f = 0.0;
    for (int e = 0; e < bb; ++e) f = f + v[e] * v[e];
    return f;
}
__global__ void fdiag_k(int64_t nr, int bb, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                        const double* __restrict__ v, double* __restrict__ fd) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    int32_t q = find_col(ci, rp[i], rp[i + 1], (int32_t)i);
    fd[i] = q >= 0 ? block_f(v + (int64_t)q * bb, bb) : 0.0;
}
// strength of the coupling at entry q = (i, j) of row i, symmetrised with (j, i)
__device__ __forceinline__ uint8_t strong_entry(int64_t i, int32_t q, int bb, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                const double* __restrict__ fd, double th4) {
    int32_t j = ci[q];
    if (j == i) return 0;
    double fij = block_f(v + (int64_t)q * bb, bb);
    bool s1 = (fij * fij) >= ((th4 * fd[i]) * fd[j]);
    bool s2 = false;
    int32_t t = find_col(ci, rp[j], rp[j + 1], (int32_t)i);
    if (t >= 0) {
        double fji = block_f(v + (int64_t)t * bb, bb);
        s2 = (fji * fji) >= ((th4 * fd[j]) * fd[i]);
    }
    return (s1 || s2) ? 1 : 0;
}

__global__ void strength_k(int64_t nr, int bb, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, const double* __restrict__ fd, double th4,
                           uint8_t* __restrict__ flags, uint8_t* __restrict__ iso) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    uint8_t any = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const uint8_t f = strong_entry(i, q, bb, rp, ci, v, fd, th4);
        flags[q] = f;
        any |= f;
    }
    iso[i] = any ? 0 : 1;
}

// the same with one wavefront per row, lanes over its entries (levels with long rows)
__global__ void __launch_bounds__(256) strength_wave_k(int64_t nr, int bb, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                       const double* __restrict__ fd, double th4,
                                                       uint8_t* __restrict__ flags, uint8_t* __restrict__ iso) {
    const int64_t i = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= nr) return;
    int any = 0;
    for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += WAVE) {
        const uint8_t f = strong_entry(i, q, bb, rp, ci, v, fd, th4);
        flags[q] = f;
        any |= f;
    }
    const uint64_t b = __ballot(any);
    if (lane == 0) iso[i] = b ? 0 : 1;
}

// state word: top 2 bits = 0 out/isolated, 1 undecided, 2 in; low 62 bits = priority
constexpr uint64_t ST_UND = 1ULL << 62, ST_IN = 2ULL << 62, KEYMASK = (1ULL << 62) - 1;

__global__ void mis_init_k(int64_t nr, const uint8_t* __restrict__ iso, uint64_t seed, int level, uint64_t* __restrict__ st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    st[i] = iso[i] ? 0ULL : (ST_UND | mis_key(seed, level, i));
}
__global__ void mis_max_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const uint8_t* __restrict__ flags, const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                          const uint64_t* __restrict__ und_only) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    if (und_only && (und_only[i] >> 62) != 1) return;
    uint64_t m = in[i];
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        if (flags[q]) {
            uint64_t v = in[ci[q]];
            m = v > m ? v : m;
        }
    out[i] = m;
}
// the same with one wavefront per row (levels with long rows)
__global__ void __launch_bounds__(256) mis_max_wave_k(int64_t nr, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, const uint8_t* __restrict__ flags,
                                                      const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                      const uint64_t* __restrict__ und_only) {
    const int64_t i = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= nr) return;
    if (und_only && (und_only[i] >> 62) != 1) return;
    uint64_t m = 0;
    for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += WAVE)
        if (flags[q]) {
            uint64_t v = in[ci[q]];
            m = v > m ? v : m;
        }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        uint64_t w = __shfl_xor(m, o, WAVE);
        m = w > m ? w : m;
    }
    if (lane == 0) {
        const uint64_t self = in[i];
        out[i] = self > m ? self : m;
    }
}
// *und becomes nonzero if a node stays undecided (one atomic per workgroup at most)
__global__ void __launch_bounds__(256) mis_decide_k(int64_t nr, uint64_t* __restrict__ st,
                                                    const uint64_t* __restrict__ m2, int* __restrict__ und) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int left = 0;
    if (i < nr) {
        uint64_t s = st[i];
        if ((s >> 62) == 1) {
            uint64_t m = m2[i];
            if ((m >> 62) == 2) st[i] = s & KEYMASK;               // an IN node within distance 2
            else if (m == s) st[i] = ST_IN | (s & KEYMASK);        // largest undecided priority within distance 2
            else left = 1;
        }
    }
    if (__syncthreads_or(left) && threadIdx.x == 0) atomicOr(und, 1);
}

__global__ void root_flag_k(int64_t nr, const uint64_t* __restrict__ st, int32_t* __restrict__ isroot) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) isroot[i] = (st[i] >> 62) == 2 ? 1 : 0;
}
__global__ void agg_roots_k(int64_t nr, const uint64_t* __restrict__ st, const int32_t* __restrict__ rid,
                            int32_t* __restrict__ agg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) agg[i] = (st[i] >> 62) == 2 ? rid[i] : -1;
}
__global__ void agg_dist1_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const uint8_t* __restrict__ flags, const uint8_t* __restrict__ iso, const uint64_t* __restrict__ st,
                            const int32_t* __restrict__ rid, int32_t* __restrict__ agg, uint8_t* __restrict__ step1) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    step1[i] = 0;
    if (iso[i] || (st[i] >> 62) == 2) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        int32_t j = ci[q];
        if (flags[q] && (st[j] >> 62) == 2) {
            agg[i] = rid[j];
            step1[i] = 1;
            return;
        }
    }
}
__global__ void agg_dist2_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const uint8_t* __restrict__ flags, const uint8_t* __restrict__ iso,
                            const uint8_t* __restrict__ step1, uint64_t seed, int level, int32_t* __restrict__ agg,
                            int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    if (iso[i] || agg[i] >= 0) return;
    uint64_t best = 0;
    int32_t bj = -1;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        int32_t j = ci[q];
        if (!flags[q] || !step1[j]) continue;
        uint64_t kj = mis_key(seed, level, j);
        if (bj < 0 || kj > best) { best = kj; bj = j; }
    }
    if (bj < 0) { atomicOr(err, 1); return; }
    agg[i] = agg[bj];   // bj joined in the distance-1 step: its aggregate is final
}

// ====================================================================== tentative prolongator
__global__ void agg_count_k(int64_t nr, const int32_t* __restrict__ agg, int32_t* __restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr && agg[i] >= 0) atomicAdd(&cnt[agg[i]], 1);
}
__global__ void agg_fill_k(int64_t nr, const int32_t* __restrict__ agg, const int32_t* __restrict__ mrp,
                           int32_t* __restrict__ fillc, int32_t* __restrict__ mem) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr && agg[i] >= 0) mem[mrp[agg[i]] + atomicAdd(&fillc[agg[i]], 1)] = (int32_t)i;
}
__global__ void agg_sort_k(int64_t na, const int32_t* __restrict__ mrp, int32_t* __restrict__ mem) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    int32_t lo = mrp[a], hi = mrp[a + 1];
    for (int32_t t = lo + 1; t < hi; ++t) {
        int32_t v = mem[t], u = t - 1;
        while (u >= lo && mem[u] > v) { mem[u + 1] = mem[u]; --u; }
        mem[u + 1] = v;
    }
}

// Gram-Schmidt (two modified-GS passes) of B restricted to the aggregate's rows (members in
// ascending order, b rows each).  Column j is dead when its remainder is <= 1e-10 of its norm.
__global__ void tentative_k(int64_t na, int b, int k, const int32_t* __restrict__ mrp, const int32_t* __restrict__ mem,
                            const double* __restrict__ B, double* __restrict__ Q, double* __restrict__ Bc,
                            uint8_t* __restrict__ dead) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    int32_t lo = mrp[a], hi = mrp[a + 1];
    double* Rk = Bc + a * k * k;
    for (int e = 0; e < k * k; ++e) Rk[e] = 0.0;
    // Q rows of the members start as B rows
    for (int32_t t = lo; t < hi; ++t) {
        int64_t node = mem[t];
        for (int r = 0; r < b; ++r)
            for (int c = 0; c < k; ++c) Q[(node * b + r) * k + c] = B[(node * b + r) * k + c];
    }
    for (int j = 0; j < k; ++j) {
        double nb = 0.0;
        for (int32_t t = lo; t < hi; ++t)
            for (int r = 0; r < b; ++r) {
                double w = Q[((int64_t)mem[t] * b + r) * k + j];
                nb += w * w;
            }
        nb = sqrt(nb);
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                if (dead[a * k + i]) continue;
                double c = 0.0;
                for (int32_t t = lo; t < hi; ++t)
                    for (int r = 0; r < b; ++r) {
                        int64_t row = ((int64_t)mem[t] * b + r) * k;
                        c += Q[row + i] * Q[row + j];
                    }
                for (int32_t t = lo; t < hi; ++t)
                    for (int r = 0; r < b; ++r) {
                        int64_t row = ((int64_t)mem[t] * b + r) * k;
                        Q[row + j] -= c * Q[row + i];
                    }
                Rk[i * k + j] += c;
            }
        double nv = 0.0;
        for (int32_t t = lo; t < hi; ++t)
            for (int r = 0; r < b; ++r) {
                double w = Q[((int64_t)mem[t] * b + r) * k + j];
                nv += w * w;
            }
        nv = sqrt(nv);
        bool isdead = (nb == 0.0) || (nv <= 1e-10 * nb);
        dead[a * k + j] = isdead ? 1 : 0;
        for (int32_t t = lo; t < hi; ++t)
            for (int r = 0; r < b; ++r) {
                int64_t row = ((int64_t)mem[t] * b + r) * k;
                Q[row + j] = isdead ? 0.0 : Q[row + j] / nv;
            }
        Rk[j * k + j] = isdead ? 0.0 : nv;
    }
}

// The same factorisation with one wavefront per aggregate and the aggregate's rows of Q in LDS
// (rows in member order, k columns).  Every sum is taken by lane 0 in that row order, so the
// rounding is that of tentative_k; the element-wise updates run on all lanes.
__global__ void __launch_bounds__(WAVE) tentative_lds_k(int64_t na, int b, int k, const int32_t* __restrict__ mrp,
                                                        const int32_t* __restrict__ mem, const double* __restrict__ B,
                                                        double* __restrict__ Q, double* __restrict__ Bc,
                                                        uint8_t* __restrict__ dead) {
    extern __shared__ double q[];
    __shared__ double bc[2];
    __shared__ double rk[64];      // R of the aggregate (k <= 8)
    __shared__ uint8_t dl[8];
    const int64_t a = blockIdx.x;
    if (a >= na) return;
    const int lane = threadIdx.x;
    const int32_t lo = mrp[a], hi = mrp[a + 1];
    const int nrow = (hi - lo) * b;
    for (int e = lane; e < nrow * k; e += WAVE) {
        const int rr = e / k, c = e - rr * k;
        const int t = rr / b, r = rr - t * b;
        q[e] = B[((int64_t)mem[lo + t] * b + r) * k + c];
    }
    for (int e = lane; e < k * k; e += WAVE) rk[e] = 0.0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        double nb = 0.0;
        if (lane == 0) {
            for (int rr = 0; rr < nrow; ++rr) nb += q[rr * k + j] * q[rr * k + j];
            nb = sqrt(nb);
        }
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                if (dl[i]) continue;           // written and synchronised when column i finished
                if (lane == 0) {
                    double c = 0.0;
                    for (int rr = 0; rr < nrow; ++rr) c += q[rr * k + i] * q[rr * k + j];
                    bc[0] = c;
                    rk[i * k + j] += c;
                }
                __syncthreads();
                const double c = bc[0];
                for (int rr = lane; rr < nrow; rr += WAVE) q[rr * k + j] -= c * q[rr * k + i];
                __syncthreads();
            }
        if (lane == 0) {
            double nv = 0.0;
            for (int rr = 0; rr < nrow; ++rr) nv += q[rr * k + j] * q[rr * k + j];
            nv = sqrt(nv);
            const bool isdead = (nb == 0.0) || (nv <= 1e-10 * nb);
            dl[j] = isdead ? 1 : 0;
            dead[a * k + j] = isdead ? 1 : 0;
            rk[j * k + j] = isdead ? 0.0 : nv;
            bc[1] = nv;
        }
        __syncthreads();
        const double nv = bc[1];
        const bool isdead = dl[j] != 0;
        for (int rr = lane; rr < nrow; rr += WAVE) q[rr * k + j] = isdead ? 0.0 : q[rr * k + j] / nv;
        __syncthreads();
    }
    for (int e = lane; e < nrow * k; e += WAVE) {
        const int rr = e / k, c = e - rr * k;
        const int t = rr / b, r = rr - t * b;
        Q[((int64_t)mem[lo + t] * b + r) * k + c] = q[e];
    }
    for (int e = lane; e < k * k; e += WAVE) Bc[a * k * k + e] = rk[e];
}

// tentative prolongator of all aggregates: the LDS form when the largest aggregate fits
static void tentative_run(int64_t na, int b, int k, const int32_t* mrp, const int32_t* mem, const double* B,
                          double* Q, double* Bc, uint8_t* dead, Arena& ar, hipStream_t s) {
    if (na <= 0) return;
    int* mx = ar.make<int>(1);
    zero_dev(mx, sizeof(int), s);
    rowlen_max_k<<<cdiv(na, 256), 256, 0, s>>>(na, mrp, mx);
    check_launch("agg_max");
    int hm = 0;
    HIPCHK(hipMemcpyAsync(&hm, mx, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(mx);
    const size_t lds = (size_t)hm * b * k * sizeof(double);
    if (k <= 8 && lds <= 48 * 1024) tentative_lds_k<<<(unsigned)na, WAVE, lds, s>>>(na, b, k, mrp, mem, B, Q, Bc, dead);
    else tentative_k<<<cdiv(na, 64), 64, 0, s>>>(na, b, k, mrp, mem, B, Q, Bc, dead);
    check_launch("tentative");
}

// P_tent as BSR: one b x k block per aggregated row
__global__ void ptent_cnt_k(int64_t nr, const int32_t* __restrict__ agg, int32_t* __restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) cnt[i] = agg[i] >= 0 ? 1 : 0;
}
__global__ void ptent_fill_k(int64_t nr, int bk, const int32_t* __restrict__ agg, const int32_t* __restrict__ rp,
                             const double* __restrict__ Q, int32_t* __restrict__ ci, double* __restrict__ v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr || agg[i] < 0) return;
    int32_t q = rp[i];
    ci[q] = agg[i];
    for (int e = 0; e < bk; ++e) v[(int64_t)q * bk + e] = Q[i * bk + e];
}

// ====================================================================== D^-1 and lambda_hat
template <int B>
__device__ bool invert_small(const double* __restrict__ a, double* __restrict__ out) {
    double m[B][2 * B];
    for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) {
            m[r][c] = a[r * B + c];
            m[r][B + c] = r == c ? 1.0 : 0.0;
        }
    for (int k = 0; k < B; ++k) {
        int p = k;
        double best = fabs(m[k][k]);
        for (int r = k + 1; r < B; ++r)
            if (fabs(m[r][k]) > best) { best = fabs(m[r][k]); p = r; }
        if (best == 0.0) return false;
        if (p != k)
            for (int c = 0; c < 2 * B; ++c) { double t = m[k][c]; m[k][c] = m[p][c]; m[p][c] = t; }
        double piv = m[k][k];
        for (int c = 0; c < 2 * B; ++c) m[k][c] /= piv;
        for (int r = 0; r < B; ++r) {
            if (r == k) continue;
            double f = m[r][k];
            for (int c = 0; c < 2 * B; ++c) m[r][c] -= f * m[k][c];
        }
    }
    for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) out[r * B + c] = m[r][B + c];
    return true;
}

template <int B>
__global__ void __launch_bounds__(256) dinv_lambda_k(int64_t nr, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                     double* __restrict__ Dinv, unsigned long long* __restrict__ lam,
                                                     int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0;     // max absolute row sum of D^-1 A over the block row (0 for idle threads)
    if (i < nr) {
        int32_t q = find_col(ci, rp[i], rp[i + 1], (int32_t)i);
        double Di[B * B];
        if (q < 0 || !invert_small<B>(v + (int64_t)q * B * B, Di)) {
            atomicOr(err, 1);
        } else {
            for (int e = 0; e < B * B; ++e) Dinv[i * B * B + e] = Di[e];
            double rs[B];
            for (int r = 0; r < B; ++r) rs[r] = 0.0;
            for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
                const double* blk = v + (int64_t)t * B * B;
                for (int r = 0; r < B; ++r)
                    for (int c = 0; c < B; ++c) {
                        double sum = 0.0;
                        for (int l = 0; l < B; ++l) sum += Di[r * B + l] * blk[l * B + c];
                        rs[r] += fabs(sum);
                    }
            }
            for (int r = 0; r < B; ++r) m = rs[r] > m ? rs[r] : m;
        }
    }
    // nonnegative doubles order as their bit patterns
    block_max_to((unsigned long long)__double_as_longlong(m), lam);
}

// P = -omega D^-1 (A P_tent) + P_tent  (rows of AP_t are those of P)
template <int B, int K>
__global__ void smooth_p_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           double* __restrict__ v, const double* __restrict__ Dinv, const int32_t* __restrict__ agg,
                           const double* __restrict__ Q, double omega) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr || agg[i] < 0) return;
    const double* Di = Dinv + i * B * B;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        double* blk = v + (int64_t)q * B * K;
        double t[B * K];
        for (int r = 0; r < B; ++r)
            for (int c = 0; c < K; ++c) {
                double sum = 0.0;
                for (int l = 0; l < B; ++l) sum += Di[r * B + l] * blk[l * K + c];
                t[r * K + c] = -omega * sum;
            }
        if (ci[q] == agg[i])
            for (int e = 0; e < B * K; ++e) t[e] += Q[i * B * K + e];
        for (int e = 0; e < B * K; ++e) blk[e] = t[e];
    }
}

// ====================================================================== transpose
__global__ void tr_count_k(int64_t nnz, const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) atomicAdd(&cnt[ci[q]], 1);
}
__global__ void tr_fill_k(int64_t nr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const int32_t* __restrict__ trp, int32_t* __restrict__ fillc, int32_t* __restrict__ tci,
                          int32_t* __restrict__ src) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        int32_t c = ci[q];
        int32_t pos = trp[c] + atomicAdd(&fillc[c], 1);
        tci[pos] = (int32_t)i;
        src[pos] = q;
    }
}
// place each entry of a transposed row at its rank (source rows are unique within a row)
__global__ void tr_rank_k(int64_t nnz, int64_t ntr, const int32_t* __restrict__ trp, const int32_t* __restrict__ tci,
                          const int32_t* __restrict__ src, const double* __restrict__ v, int br, int bc,
                          int32_t* __restrict__ oci, double* __restrict__ ov, const int32_t* __restrict__ rowof) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    int32_t r = rowof[p];
    int32_t lo = trp[r], hi = trp[r + 1];
    int32_t key = tci[p], rank = 0;
    for (int32_t u = lo; u < hi; ++u) rank += tci[u] < key;
    int64_t dst = lo + rank;
    oci[dst] = key;
    const double* s = v + (int64_t)src[p] * br * bc;
    double* d = ov + dst * br * bc;
    for (int r0 = 0; r0 < br; ++r0)
        for (int c0 = 0; c0 < bc; ++c0) d[c0 * br + r0] = s[r0 * bc + c0];
}
__global__ void row_of_k(int64_t nr, const int32_t* __restrict__ rp, int32_t* __restrict__ rowof) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) rowof[q] = (int32_t)i;
}

DBsr transpose(const DBsr& M, Arena& ar, hipStream_t s) {
    DBsr T;
    T.nr = M.nc; T.nc = M.nr; T.br = M.bc; T.bc = M.br; T.nnzb = M.nnzb;
    int32_t* cnt = ar.make<int32_t>(M.nc + 1);
    zero_dev(cnt, (M.nc + 1) * sizeof(int32_t), s);
    if (M.nnzb) tr_count_k<<<cdiv(M.nnzb, 256), 256, 0, s>>>(M.nnzb, M.ci, cnt);
    T.rp = ar.make<int32_t>(M.nc + 1);
    scan_i32(cnt, T.rp, M.nc, ar, s);
    zero_dev(cnt, (M.nc + 1) * sizeof(int32_t), s);
    int32_t* tci = ar.make<int32_t>(M.nnzb + 1);
    int32_t* src = ar.make<int32_t>(M.nnzb + 1);
    if (M.nr) tr_fill_k<<<cdiv(M.nr, 256), 256, 0, s>>>(M.nr, M.rp, M.ci, T.rp, cnt, tci, src);
    int32_t* rowof = ar.make<int32_t>(M.nnzb + 1);
    if (T.nr) row_of_k<<<cdiv(T.nr, 256), 256, 0, s>>>(T.nr, T.rp, rowof);
    T.ci = ar.make<int32_t>(M.nnzb + 1);
    T.v = ar.make<double>((M.nnzb + 1) * M.br * M.bc);
    if (M.nnzb)
        tr_rank_k<<<cdiv(M.nnzb, 256), 256, 0, s>>>(M.nnzb, T.nr, T.rp, tci, src, M.v, M.br, M.bc, T.ci, T.v, rowof);
    check_launch("transpose");
    ar.free(cnt); ar.free(tci); ar.free(src); ar.free(rowof);
    return T;
}

__global__ void dead_diag_k(int64_t na, int k, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            double* __restrict__ v, const uint8_t* __restrict__ dead) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    int32_t q = find_col(ci, rp[a], rp[a + 1], (int32_t)a);
    if (q < 0) return;
    for (int c = 0; c < k; ++c)
        if (dead[a * k + c]) v[(int64_t)q * k * k + c * k + c] = 1.0;
}

// ====================================================================== coarsest level: dense inverse
__global__ void densify_k(int64_t nr, int b, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ v, double* __restrict__ M, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q)
        for (int r = 0; r < b; ++r)
            for (int c = 0; c < b; ++c) M[(i * b + r) * n + (int64_t)ci[q] * b + c] = v[((int64_t)q * b + r) * b + c];
}
// Gauss-Jordan exchange steps over all pivots in order turn A into A^-1.  This fast form takes
// the pivots in order without interchanges; the result is checked afterwards (the backward error
// of one solve with it, coarse_check_*) and recomputed with row interchanges (partial pivoting,
// gjp_*) when a small or zero leading pivot spoilt it: the coarsest operators are not SPD in
// general (the advective velocity block is nonsymmetric).
// A panel of GJ_P consecutive pivots K = [k0, k0 + np) at once, by the block form of the exchange
// step (equal in exact arithmetic to the np single steps in order): with W = M_KK^-1,
//   out_KK = W,  out_KR = W M_KR,  out_RK = -M_RK W,  out_RR = M_RR - M_RK W M_KR.
constexpr int GJ_P = 32;
// W by single exchange steps in LDS (every workgroup, redundantly), then T = M_RK W for the
// workgroup's rows (T is n x GJ_P); workgroup 0 also stores W
__global__ void __launch_bounds__(256) gj_panel_t_k(int64_t n, int64_t k0, int np, const double* __restrict__ src,
                                                    double* __restrict__ T, double* __restrict__ Wout) {
    __shared__ double W[GJ_P][GJ_P + 1];
    constexpr int PER = GJ_P * GJ_P / 256;     // entries of W per thread (compile-time: registers)
    {
        double w0[PER];     // all loads issued before the first is used (clamped, branch-free indices)
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            int e = threadIdx.x + 256 * c;
            int ee = e < np * np ? e : 0;
            w0[c] = src[(k0 + ee / np) * n + k0 + ee % np];
        }
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            int e = threadIdx.x + 256 * c;
            if (e < np * np) W[e / np][e % np] = w0[c];
        }
    }
    __syncthreads();
    for (int k = 0; k < np; ++k) {
        const double ip = 1.0 / W[k][k];
        double upd[PER];
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            int e = threadIdx.x + 256 * c;
            upd[c] = 0.0;
            if (e < np * np) {
                int i = e / np, j = e % np;
                if (i == k) upd[c] = (j == k) ? ip : W[k][j] * ip;
                else if (j == k) upd[c] = -W[i][k] * ip;
                else upd[c] = W[i][j] - W[i][k] * W[k][j] * ip;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            int e = threadIdx.x + 256 * c;
            if (e < np * np) W[e / np][e % np] = upd[c];
        }
        __syncthreads();
    }
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < np * np; e += 256) Wout[e] = W[e / np][e % np];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double r[GJ_P];     // the row's panel entries, loaded once (clamped, branch-free indices)
#pragma unroll
    for (int l = 0; l < GJ_P; ++l) r[l] = src[i * n + k0 + (l < np ? l : np - 1)];
    for (int c = 0; c < np; ++c) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < GJ_P; ++l)
            if (l < np) t += r[l] * W[l][c];
        T[i * GJ_P + c] = t;
    }
}
__global__ void gj_panel_apply_k(int64_t n, int64_t k0, int np, const double* __restrict__ src,
                                 const double* __restrict__ T, const double* __restrict__ W, double* __restrict__ dst) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int64_t i = idx / n, j = idx % n;
    bool iK = i >= k0 && i < k0 + np, jK = j >= k0 && j < k0 + np;
    double out;
    if (iK && jK) {
        out = W[(i - k0) * np + (j - k0)];
    } else if (iK) {
        out = 0.0;
        for (int l = 0; l < np; ++l) out += W[(i - k0) * np + l] * src[(k0 + l) * n + j];
    } else if (jK) {
        out = -T[i * GJ_P + (j - k0)];
    } else {
        out = src[idx];
        for (int l = 0; l < np; ++l) out -= T[i * GJ_P + l] * src[(k0 + l) * n + j];
    }
    dst[idx] = out;
}
__global__ void finite_k(int64_t n, const double* __restrict__ a, int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(err, 1);
}

// ---- accuracy check of an explicit inverse X of A: y = X v for a fixed v, then the normwise
// backward error eta = ||A y - v||_inf / (||A||_inf ||y||_inf + ||v||_inf) (about n * 1e-16 for
// a stable inverse; a spoilt pivot makes it large or non-finite)
__device__ __forceinline__ double check_vec(int64_t i) { return 1.0 + (double)((i * 7919) % 13) / 13.0; }
__global__ void __launch_bounds__(256) coarse_check_y_k(int64_t n, const double* __restrict__ X, double* __restrict__ y) {
    int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (row >= n) return;
    int lane = threadIdx.x & (WAVE - 1);
    double acc = 0.0;
    for (int64_t c = lane; c < n; c += WAVE) acc += X[row * n + c] * check_vec(c);
    acc = wave_sum(acc);
    if (lane == 0) y[row] = acc;
}
// per row: |(A y)_i - v_i| and the absolute row sum of A
__global__ void __launch_bounds__(256) coarse_check_r_k(int64_t n, const double* __restrict__ A, const double* __restrict__ y,
                                                        double* __restrict__ rr, double* __restrict__ ra) {
    int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (row >= n) return;
    int lane = threadIdx.x & (WAVE - 1);
    double acc = 0.0, abs_sum = 0.0;
    for (int64_t c = lane; c < n; c += WAVE) {
        acc += A[row * n + c] * y[c];
        abs_sum += fabs(A[row * n + c]);
    }
    acc = wave_sum(acc);
    abs_sum = wave_sum(abs_sum);
    if (lane == 0) {
        rr[row] = fabs(acc - check_vec(row));
        ra[row] = abs_sum;
    }
}
// one workgroup: eta into *eta (NaN propagates: fmax would drop it, so non-finite values are flagged)
__global__ void __launch_bounds__(256) coarse_check_eta_k(int64_t n, const double* __restrict__ rr,
                                                          const double* __restrict__ ra, const double* __restrict__ y,
                                                          double* __restrict__ eta) {
    __shared__ double red[3][256];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    double m[3] = {0.0, 0.0, 0.0};
    int nf = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double a = rr[i], b = ra[i], c = fabs(y[i]);
        if (!isfinite(a) || !isfinite(b) || !isfinite(c)) nf = 1;
        m[0] = a > m[0] ? a : m[0];
        m[1] = b > m[1] ? b : m[1];
        m[2] = c > m[2] ? c : m[2];
    }
    if (nf) atomicOr(&bad, 1);
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *eta = bad ? INFINITY : red[0][0] / (red[1][0] * red[2][0] + 2.0);
}

// ---- Gauss-Jordan with partial pivoting (the fallback): step k picks the row p >= k with the
// largest |M_pk| (the smallest such p on ties), swaps rows k and p of the current matrix and
// applies the exchange step at (k, k); at the end the column interchanges are undone in reverse
// order (the inverse of the row-permuted matrix is A^-1 P^-1).
__global__ void __launch_bounds__(256) gjp_pivot_k(int64_t n, int64_t k, double* __restrict__ M, int32_t* __restrict__ perm,
                                                   int* __restrict__ err) {
    __shared__ double bv[256];
    __shared__ int64_t bi[256];
    double best = -1.0;
    int64_t arg = n;
    for (int64_t i = k + threadIdx.x; i < n; i += 256) {
        const double v = fabs(M[i * n + k]);
        if (v > best) { best = v; arg = i; }     // ascending i per thread: the first largest
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = arg;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double v = bv[threadIdx.x + o];
            const int64_t a = bi[threadIdx.x + o];
            if (v > bv[threadIdx.x] || (v == bv[threadIdx.x] && a < bi[threadIdx.x])) {
                bv[threadIdx.x] = v;
                bi[threadIdx.x] = a;
            }
        }
        __syncthreads();
    }
    const int64_t p = bi[0];
    if (threadIdx.x == 0) {
        perm[k] = (int32_t)(p < n ? p : k);
        if (!(bv[0] > 0.0) || !isfinite(bv[0])) atomicOr(err, 1);
    }
    if (p >= n || p == k) return;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double a = M[k * n + j];
        M[k * n + j] = M[p * n + j];
        M[p * n + j] = a;
    }
}
__global__ void gjp_exchange_k(int64_t n, int64_t k, const double* __restrict__ src, double* __restrict__ dst) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int64_t i = idx / n, j = idx % n;
    const double ip = 1.0 / src[k * n + k];
    double out;
    if (i == k) out = (j == k) ? ip : src[k * n + j] * ip;
    else if (j == k) out = -src[i * n + k] * ip;
    else out = src[idx] - src[i * n + k] * src[k * n + j] * ip;
    dst[idx] = out;
}
// undo the interchanges on the columns: row i applies swap (k, perm[k]) for k = n-1 .. 0
__global__ void gjp_unpermute_k(int64_t n, const int32_t* __restrict__ perm, double* __restrict__ M) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* row = M + i * n;
    for (int64_t k = n - 1; k >= 0; --k) {
        const int64_t p = perm[k];
        if (p != k) {
            const double a = row[k];
            row[k] = row[p];
            row[p] = a;
        }
    }
}

// ====================================================================== hierarchy with solve-phase data in T
template <typename T>
class HierT : public Hierarchy {
   public:
    struct LS {
        DSell<T> A, P;
        DBsrT<T> R;
        T* Dinv = nullptr;
        T *b = nullptr, *x = nullptr, *w = nullptr, *t1 = nullptr, *t2 = nullptr, *d = nullptr, *r = nullptr;
        // the same vectors for three interleaved columns (scalar hierarchies built with `three`)
        T *b3 = nullptr, *x3 = nullptr, *w3 = nullptr, *t13 = nullptr, *t23 = nullptr, *d3 = nullptr, *r3 = nullptr;
        std::vector<double> c1, c2;    // smoothing-step coefficients
        bool cheb = false;
    };
    std::vector<LS> S;
    Arena* ar = nullptr;
    Profiler* prof = nullptr;

    void prepare(Arena& a, hipStream_t s) {
        ar = &a;
        S.resize(L.size());
        for (size_t l = 0; l < L.size(); ++l) {
            LevelSetup& ls = L[l];
            LS& q = S[l];
            int64_t n = ls.A.nr * ls.b;
            q.b = a.make<T>(n); q.x = a.make<T>(n);
            if (three) { q.b3 = a.make<T>(3 * n); q.x3 = a.make<T>(3 * n); }
            if (l + 1 == L.size()) continue;
            q.A = sell_from_bsr<T>(ls.A, a, s);
            q.P = sell_from_bsr<T>(ls.P, a, s);
            q.R = bsrt_from_bsr<T>(ls.R, a, s);
            int64_t bb = (int64_t)ls.A.nr * ls.b * ls.b;
            q.Dinv = a.make<T>(bb);
            if (std::is_same<T, double>::value) copy_d(bb, ls.Dinv, (double*)q.Dinv, s);
            else cast_d2f(ls.Dinv, (float*)q.Dinv, bb, s);
            q.w = a.make<T>(n); q.t1 = a.make<T>(n); q.t2 = a.make<T>(n); q.d = a.make<T>(n); q.r = a.make<T>(n);
            if (three) {
                q.w3 = a.make<T>(3 * n); q.t13 = a.make<T>(3 * n); q.t23 = a.make<T>(3 * n);
                q.d3 = a.make<T>(3 * n); q.r3 = a.make<T>(3 * n);
            }
            // smoothing coefficients: step t computes dn = c1[t] d + c2[t] Dinv (b - A x)
            if (opts.smoother == SCR_SMOOTH_CHEBYSHEV) {
                q.cheb = true;
                double lmax = ls.lam, lmin = ls.lam / opts.cheb_ratio;
                double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
                double sigma = theta / delta, rho_prev = 1.0 / sigma;
                q.c1.push_back(0.0); q.c2.push_back(1.0 / theta);
                for (int t = 1; t < opts.cheb_degree; ++t) {
                    double rho = 1.0 / (2.0 * sigma - rho_prev);
                    q.c1.push_back(rho * rho_prev); q.c2.push_back(2.0 * rho / delta);
                    rho_prev = rho;
                }
            } else {
                double w = 4.0 / (3.0 * ls.lam);
                for (int t = 0; t < opts.jacobi_sweeps; ++t) { q.c1.push_back(0.0); q.c2.push_back(w); }
            }
        }
    }

    void refresh(Arena& a, hipStream_t s) override {
        for (auto& q : S) {
            sell_free(q.A, a);
            sell_free(q.P, a);
            a.free(q.R.v);
            for (T* p : {q.Dinv, q.b, q.x, q.w, q.t1, q.t2, q.d, q.r}) a.free(p);
            for (T* p : {q.b3, q.x3, q.w3, q.t13, q.t23, q.d3, q.r3}) a.free(p);
        }
        S.clear();
        prepare(a, s);
    }

    // algorithmic bytes of one smoother step with a matrix product: every stored block (values
    // and column index) once, a 4-byte row index per block row, x once, the right-hand side, the
    // output and d as used.  D^-1 is not counted: it follows from the diagonal block the step
    // streams anyway (the block-row-lane kernels solve with that block; the other smoothers read
    // the stored inverse, which this count leaves out).
    double step_bytes(const LS& q, bool rd, bool wd) const {
        const double b = q.A.br, t = sizeof(T);
        double rows = (double)q.A.nr;
        return (double)q.A.nnzb * (b * b * t + 4.0) + rows * (4.0 + b * t * (3.0 + (rd ? 1.0 : 0.0) + (wd ? 1.0 : 0.0)));
    }

    // smoothing sweeps from xin (nullptr = zero) into dst
    void smooth(size_t l, LS& q, const T* b, const T* xin, T* dst, hipStream_t s) {
        int ns = (int)q.c1.size();
        const T* cur = xin;
        for (int t = 0; t < ns; ++t) {
            T* out = (t == ns - 1) ? dst : ((t % 2 == 0) ? q.t1 : q.t2);
            bool rd = q.cheb && t > 0, wd = q.cheb && t + 1 < ns, zero = cur == nullptr;
            bool timed = prof && l == 0 && !zero;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) { e0 = prof->get(); e1 = prof->get(); }
            smooth_step<T>(q.A, q.Dinv, b, cur, q.d, out, q.c1[t], q.c2[t], rd, wd, zero, s, e0, e1);
            if (timed) prof->push(e0, e1, step_bytes(q, rd, wd));
            cur = out;
        }
    }

    void cycle(size_t l, const T* b, T* x, hipStream_t s) {
        if (l + 1 == S.size()) {
            dense_mv<T>(ncoarse, cinv, b, x, s);
            return;
        }
        LS& q = S[l];
        smooth(l, q, b, nullptr, q.w, s);
        sell_mv<T>(q.A, q.w, b, q.r, 1, s);
        bsrt_mv<T>(q.R, q.r, S[l + 1].b, s);
        cycle(l + 1, S[l + 1].b, S[l + 1].x, s);
        sell_mv<T>(q.P, S[l + 1].x, nullptr, q.w, 2, s);
        smooth(l, q, b, q.w, x, s);
    }

    // the V-cycle on three interleaved columns: every kernel passes over its matrix once for all
    // three, and each column's result is bitwise the one-column V-cycle's
    void smooth3(LS& q, const T* b, const T* xin, T* dst, hipStream_t s) {
        int ns = (int)q.c1.size();
        const T* cur = xin;
        for (int t = 0; t < ns; ++t) {
            T* out = (t == ns - 1) ? dst : ((t % 2 == 0) ? q.t13 : q.t23);
            bool rd = q.cheb && t > 0, wd = q.cheb && t + 1 < ns, zero = cur == nullptr;
            smooth_step3<T>(q.A, q.Dinv, b, cur, q.d3, out, q.c1[t], q.c2[t], rd, wd, zero, s);
            cur = out;
        }
    }
    void cycle3(size_t l, const T* b, T* x, hipStream_t s) {
        if (l + 1 == S.size()) {
            dense_mv3<T>(ncoarse, cinv, b, x, s);
            return;
        }
        LS& q = S[l];
        smooth3(q, b, nullptr, q.w3, s);
        sell_mv3<T>(q.A, q.w3, b, q.r3, 1, s);
        bsrt_mv3<T>(q.R, q.r3, S[l + 1].b3, s);
        cycle3(l + 1, S[l + 1].b3, S[l + 1].x3, s);
        sell_mv3<T>(q.P, S[l + 1].x3, nullptr, q.w3, 2, s);
        smooth3(q, b, q.w3, x, s);
    }
    void vcycle3(const double* x, double* y, hipStream_t s) override {
        if (!three) throw Error(SCR_E_INVALID, "three-column V-cycle on a hierarchy built without it");
        vcycles += 3;
        int64_t n = n0();
        if (std::is_same<T, double>::value) {
            cycle3(0, (const T*)x, (T*)y, s);
        } else {
            cast_d2f(x, (float*)S[0].b3, 3 * n, s);
            cycle3(0, S[0].b3, S[0].x3, s);
            cast_f2d((const float*)S[0].x3, y, 3 * n, s);
        }
    }

    void vcycle_f(const float* x, float* y, hipStream_t s) override {
        if (!std::is_same<T, float>::value) throw Error(SCR_E_INVALID, "FP32 V-cycle on an FP64 hierarchy");
        ++vcycles;
        cycle(0, (const T*)x, (T*)y, s);
    }
    const DSell<float>* level0_f() const override {
        if (!std::is_same<T, float>::value || S.size() < 2) return nullptr;
        return (const DSell<float>*)&S[0].A;
    }

    void vcycle(const double* x, double* y, hipStream_t s) override {
        ++vcycles;
        int64_t n = n0();
        if (std::is_same<T, double>::value) {
            cycle(0, (const T*)x, (T*)y, s);
        } else {
            cast_d2f(x, (float*)S[0].b, n, s);
            cycle(0, S[0].b, S[0].x, s);
            cast_f2d((const float*)S[0].x, y, n, s);
        }
    }
};

__global__ void rowmask_k(int64_t nr, const int32_t* __restrict__ agg, uint8_t* __restrict__ m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) m[i] = agg[i] >= 0 ? 1 : 0;
}

// ====================================================================== hierarchy construction
static int64_t read_i32(const int32_t* p, hipStream_t s) {
    int32_t v = 0;
    HIPCHK(hipMemcpyAsync(&v, p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return v;
}

// D^-1 (into L.Dinv) and lambda_hat = max abs row sum of D^-1 A (into L.lam)
void level_diag(LevelSetup& L, int l, int* err, unsigned long long* lamd, hipStream_t s) {
    const int64_t nr = L.A.nr;
    const int64_t g = cdiv(nr, 256);
    const int b = L.b;
    zero_dev(err, sizeof(int), s);
    zero_dev(lamd, sizeof(unsigned long long), s);
    if (g) {
        if (b == 1) dinv_lambda_k<1><<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.A.v, L.Dinv, lamd, err);
        else if (b == 3) dinv_lambda_k<3><<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.A.v, L.Dinv, lamd, err);
        else if (b == 6) dinv_lambda_k<6><<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.A.v, L.Dinv, lamd, err);
        else throw Error(SCR_E_UNIMPLEMENTED, "AMG block size");
    }
    check_launch("dinv_lambda");
    unsigned long long hl = 0;
    int he = 0;
    HIPCHK(hipMemcpyAsync(&hl, lamd, sizeof(hl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&he, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (he) throw Error(SCR_E_INVALID, "singular or missing diagonal block at AMG level " + std::to_string(l));
    double lam;
    std::memcpy(&lam, &hl, sizeof(double));
    L.lam = lam;
}

// backward error of the explicit inverse X of the dense A (one check solve; synchronises)
static double coarse_check(int64_t nc, const double* A, const double* X, Arena& ar, hipStream_t s) {
    double* y = ar.make<double>(nc);
    double* rr = ar.make<double>(nc);
    double* ra = ar.make<double>(nc);
    double* eta = ar.make<double>(1);
    coarse_check_y_k<<<cdiv(nc, 4), 256, 0, s>>>(nc, X, y);
    coarse_check_r_k<<<cdiv(nc, 4), 256, 0, s>>>(nc, A, y, rr, ra);
    coarse_check_eta_k<<<1, 256, 0, s>>>(nc, rr, ra, y, eta);
    check_launch("coarse check");
    double he = 0.0;
    HIPCHK(hipMemcpyAsync(&he, eta, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ar.free(y); ar.free(rr); ar.free(ra); ar.free(eta);
    return he;
}

// largest accepted backward error of the fast inverse (a stable inverse gives about n * 1e-16)
constexpr double COARSE_ETA_MAX = 1e-10;

// coarsest level: explicit inverse by Gauss-Jordan exchange steps, in order (fast panels), or
// with partial pivoting when the fast inverse fails its check.  H.coarse_pivoted records which.
void coarse_inverse(Hierarchy& H, int* err, Arena& ar, hipStream_t s) {
    LevelSetup& C = H.L.back();
    int64_t nc = C.A.nr * C.b;
    H.ncoarse = nc;
    if (nc > 8192) throw Error(SCR_E_INVALID, "coarsest AMG level too large for a direct solve (" + std::to_string(nc) + ")");
    if (H.cinv) { ar.free(H.cinv); H.cinv = nullptr; }
    double* A = ar.make<double>(nc * nc + 1);      // the dense coarsest matrix, kept for the check
    double* M0 = ar.make<double>(nc * nc + 1);
    double* M1 = ar.make<double>(nc * nc + 1);
    zero_dev(A, nc * nc * sizeof(double), s);
    if (C.A.nr) densify_k<<<cdiv(C.A.nr, 256), 256, 0, s>>>(C.A.nr, C.b, C.A.rp, C.A.ci, C.A.v, A, nc);
    copy_dev(M0, A, nc * nc * sizeof(double), s);
    double* T = ar.make<double>(nc * GJ_P + 1);
    double* W = ar.make<double>(GJ_P * GJ_P);
    for (int64_t k0 = 0; k0 < nc; k0 += GJ_P) {
        int np = (int)std::min<int64_t>(GJ_P, nc - k0);
        gj_panel_t_k<<<cdiv(nc, 256), 256, 0, s>>>(nc, k0, np, M0, T, W);
        gj_panel_apply_k<<<cdiv(nc * nc, 256), 256, 0, s>>>(nc, k0, np, M0, T, W, M1);
        std::swap(M0, M1);
    }
    check_launch("coarse inverse");
    ar.free(T);
    ar.free(W);
    H.coarse_eta = nc ? coarse_check(nc, A, M0, ar, s) : 0.0;
    H.coarse_pivoted = false;
    if (!(H.coarse_eta <= COARSE_ETA_MAX)) {
        // partial pivoting, one exchange step per pivot
        int32_t* perm = ar.make<int32_t>(nc);
        zero_dev(err, sizeof(int), s);
        copy_dev(M0, A, nc * nc * sizeof(double), s);
        for (int64_t k = 0; k < nc; ++k) {
            gjp_pivot_k<<<1, 256, 0, s>>>(nc, k, M0, perm, err);
            gjp_exchange_k<<<cdiv(nc * nc, 256), 256, 0, s>>>(nc, k, M0, M1);
            std::swap(M0, M1);
        }
        gjp_unpermute_k<<<cdiv(nc, 256), 256, 0, s>>>(nc, perm, M0);
        check_launch("coarse inverse (pivoted)");
        int he = 0;
        HIPCHK(hipMemcpyAsync(&he, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ar.free(perm);
        if (he) throw Error(SCR_E_INVALID, "coarsest AMG matrix is singular");
        H.coarse_eta = coarse_check(nc, A, M0, ar, s);
        H.coarse_pivoted = true;
    }
    zero_dev(err, sizeof(int), s);
    if (nc) finite_k<<<cdiv(nc * nc, 256), 256, 0, s>>>(nc * nc, M0, err);
    int he = 0;
    HIPCHK(hipMemcpyAsync(&he, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (he) throw Error(SCR_E_INVALID, "coarsest AMG matrix is singular");
    ar.free(M1);
    ar.free(A);
    H.cinv = M0;
}

std::unique_ptr<Hierarchy> build_hierarchy(const DBsr& A0, const double* B0, int k, const scr_amg_opts& o, Arena& ar,
                                           hipStream_t s, Profiler* prof, bool three) {
    if (three && A0.br != 1) throw Error(SCR_E_INVALID, "three-column V-cycles need a scalar matrix");
    if (o.amg_type == SCR_AMG_CLASSICAL) return build_classical(A0, o, ar, s, three);
    std::unique_ptr<Hierarchy> H;
    HierT<double>* hd = nullptr;
    HierT<float>* hf = nullptr;
    if (o.precision != SCR_FP64) { hf = new HierT<float>(); hf->prof = prof; H.reset(hf); }
    else { hd = new HierT<double>(); hd->prof = prof; H.reset(hd); }
    H->opts = o;
    H->three = three;
    int* err = ar.make<int>(1);
    unsigned long long* lamd = ar.make<unsigned long long>(1);
    // level 0: copy of A0 and B0
    {
        LevelSetup l0;
        l0.A = bsr_alloc(A0.nr, A0.nc, A0.br, A0.bc, A0.nnzb, ar);
        copy_dev(l0.A.rp, A0.rp, (A0.nr + 1) * sizeof(int32_t), s);
        copy_dev(l0.A.ci, A0.ci, A0.nnzb * sizeof(int32_t), s);
        copy_dev(l0.A.v, A0.v, A0.nnzb * A0.br * A0.bc * sizeof(double), s);
        l0.b = A0.br; l0.k = k;
        l0.B = ar.make<double>(A0.nr * A0.br * k);
        copy_dev(l0.B, B0, A0.nr * A0.br * k * sizeof(double), s);
        H->L.push_back(l0);
    }
    for (int l = 0;; ++l) {
        LevelSetup& L = H->L[l];
        const int64_t nr = L.A.nr;
        const int b = L.b, bb = b * b;
        const int64_t n = nr * b;
        const int64_t g = cdiv(nr, 256);
        // D^-1 and lambda_hat (every level but the coarsest needs them; computed here for all)
        L.Dinv = ar.make<double>(nr * bb);
        level_diag(L, l, err, lamd, s);
        int he = 0;
        if (n <= o.coarse_max || l + 1 >= o.max_levels || l + 1 >= 16) break;
        // strength
        double* fd = ar.make<double>(nr);
        L.strong = ar.make<uint8_t>(L.A.nnzb > 0 ? L.A.nnzb : 1);
        uint8_t* iso = ar.make<uint8_t>(nr);
        fdiag_k<<<g, 256, 0, s>>>(nr, bb, L.A.rp, L.A.ci, L.A.v, fd);
        double theta = std::ldexp(o.theta, -l);
        double th4 = ((theta * theta) * theta) * theta;
        // rows of 16 or more entries on average: one wavefront per row (same flags)
        const bool wide = L.A.nnzb >= 16 * nr;
        if (wide) strength_wave_k<<<cdiv(nr, 256 / WAVE), 256, 0, s>>>(nr, bb, L.A.rp, L.A.ci, L.A.v, fd, th4, L.strong, iso);
        else strength_k<<<g, 256, 0, s>>>(nr, bb, L.A.rp, L.A.ci, L.A.v, fd, th4, L.strong, iso);
        check_launch("strength");
        ar.free(fd);
        // MIS-2 rounds
        uint64_t* st = ar.make<uint64_t>(nr);
        uint64_t* m1 = ar.make<uint64_t>(nr);
        uint64_t* m2 = ar.make<uint64_t>(nr);
        int* und = ar.make<int>(1);
        mis_init_k<<<g, 256, 0, s>>>(nr, iso, o.seed, l, st);
        for (int round = 0;; ++round) {
            if (round > 100000) throw Error(SCR_E_HIP, "MIS-2 did not terminate");
            zero_dev(und, sizeof(int), s);
            // the second sweep only for the undecided nodes: the decision reads nothing else of m2
            if (wide) {
                mis_max_wave_k<<<cdiv(nr, 256 / WAVE), 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.strong, st, m1, nullptr);
                mis_max_wave_k<<<cdiv(nr, 256 / WAVE), 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.strong, m1, m2, st);
            } else {
                mis_max_k<<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.strong, st, m1, nullptr);
                mis_max_k<<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.strong, m1, m2, st);
            }
            mis_decide_k<<<g, 256, 0, s>>>(nr, st, m2, und);
            check_launch("mis2");
            int hu = 0;
            HIPCHK(hipMemcpyAsync(&hu, und, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hu == 0) break;
        }
        ar.free(m1); ar.free(m2); ar.free(und);
        // aggregates
        int32_t* isroot = ar.make<int32_t>(nr + 1);
        int32_t* rid = ar.make<int32_t>(nr + 1);
        root_flag_k<<<g, 256, 0, s>>>(nr, st, isroot);
        int64_t na = scan_i32(isroot, rid, nr, ar, s);
        ar.free(isroot);
        L.agg = ar.make<int32_t>(nr);
        uint8_t* step1 = ar.make<uint8_t>(nr);
        agg_roots_k<<<g, 256, 0, s>>>(nr, st, rid, L.agg);
        agg_dist1_k<<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.strong, iso, st, rid, L.agg, step1);
        zero_dev(err, sizeof(int), s);
        agg_dist2_k<<<g, 256, 0, s>>>(nr, L.A.rp, L.A.ci, L.strong, iso, step1, o.seed, l, L.agg, err);
        check_launch("aggregate");
        HIPCHK(hipMemcpyAsync(&he, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ar.free(step1); ar.free(rid); ar.free(st); ar.free(iso);
        if (he) throw Error(SCR_E_HIP, "aggregation left a node unassigned");
        if (na <= 0 || (double)(na * L.k) > o.max_coarse_ratio * (double)n) {
            ar.free(L.agg); L.agg = nullptr;
            ar.free(L.strong); L.strong = nullptr;
            break;
        }
        L.nagg = na;
        const int kk = L.k;
        // members of each aggregate, ascending
        int32_t* mcnt = ar.make<int32_t>(na + 1);
        zero_dev(mcnt, (na + 1) * sizeof(int32_t), s);
        agg_count_k<<<g, 256, 0, s>>>(nr, L.agg, mcnt);
        int32_t* mrp = ar.make<int32_t>(na + 1);
        int64_t nmem = scan_i32(mcnt, mrp, na, ar, s);
        zero_dev(mcnt, (na + 1) * sizeof(int32_t), s);
        int32_t* mem = ar.make<int32_t>(nmem + 1);
        agg_fill_k<<<g, 256, 0, s>>>(nr, L.agg, mrp, mcnt, mem);
        agg_sort_k<<<cdiv(na, 64), 64, 0, s>>>(na, mrp, mem);
        // tentative prolongator and coarse near-null space
        double* Q = ar.make<double>(nr * b * kk);
        zero_dev(Q, nr * b * kk * sizeof(double), s);
        LevelSetup N;
        N.b = kk; N.k = kk;
        N.B = ar.make<double>(na * kk * kk);
        L.dead = ar.make<uint8_t>(na * kk);
        zero_dev(L.dead, na * kk, s);
        tentative_run(na, b, kk, mrp, mem, L.B, Q, N.B, L.dead, ar, s);
        ar.free(mcnt);
        L.mrp = mrp;
        L.mem = mem;
        DBsr Pt;
        Pt.nr = nr; Pt.nc = na; Pt.br = b; Pt.bc = kk;
        Pt.rp = ar.make<int32_t>(nr + 1);
        int32_t* pc = ar.make<int32_t>(nr + 1);
        ptent_cnt_k<<<g, 256, 0, s>>>(nr, L.agg, pc);
        Pt.nnzb = scan_i32(pc, Pt.rp, nr, ar, s);
        ar.free(pc);
        Pt.ci = ar.make<int32_t>(Pt.nnzb + 1);
        Pt.v = ar.make<double>((Pt.nnzb + 1) * b * kk);
        ptent_fill_k<<<g, 256, 0, s>>>(nr, b * kk, L.agg, Pt.rp, Q, Pt.ci, Pt.v);
        check_launch("ptent");
        // smoothed prolongator on the pattern of A * P_tent (aggregated rows only)
        uint8_t* rowmask = ar.make<uint8_t>(nr);
        rowmask_k<<<g, 256, 0, s>>>(nr, L.agg, rowmask);
        DBsr P = spgemm(L.A, Pt, rowmask, ar, s);
        ar.free(rowmask);
        bsr_release(Pt, ar);
        double omega = 4.0 / (3.0 * L.lam);
        if (b == 1 && kk == 1) smooth_p_k<1, 1><<<g, 256, 0, s>>>(nr, P.rp, P.ci, P.v, L.Dinv, L.agg, Q, omega);
        else if (b == 3 && kk == 6) smooth_p_k<3, 6><<<g, 256, 0, s>>>(nr, P.rp, P.ci, P.v, L.Dinv, L.agg, Q, omega);
        else if (b == 6 && kk == 6) smooth_p_k<6, 6><<<g, 256, 0, s>>>(nr, P.rp, P.ci, P.v, L.Dinv, L.agg, Q, omega);
        else throw Error(SCR_E_UNIMPLEMENTED, "prolongator block shape");
        check_launch("smooth_p");
        ar.free(Q);
        L.P = P;
        L.R = transpose(L.P, ar, s);
        // Galerkin product A_c = R (A P) on structural patterns; dead coarse dofs get a unit diagonal
        DBsr AP = spgemm(L.A, L.P, nullptr, ar, s);
        N.A = spgemm(L.R, AP, nullptr, ar, s);
        ar.free(AP.v);
        AP.v = nullptr;
        L.AP = AP;
        if (na) dead_diag_k<<<cdiv(na, 256), 256, 0, s>>>(na, kk, N.A.rp, N.A.ci, N.A.v, L.dead);
        check_launch("dead_diag");
        H->L.push_back(N);   // invalidates L
    }
    coarse_inverse(*H, err, ar, s);
    ar.free(err);
    ar.free(lamd);
    if (hf) hf->prepare(ar, s);
    else hd->prepare(ar, s);
    HIPCHK(hipStreamSynchronize(s));
    return H;
}

void update_hierarchy(Hierarchy& H, const double* vals0, const double* B0, Arena& ar, hipStream_t s) {
    if (H.opts.amg_type == SCR_AMG_CLASSICAL) {
        update_classical(H, vals0, ar, s);
        return;
    }
    int* err = ar.make<int>(1);
    unsigned long long* lamd = ar.make<unsigned long long>(1);
    LevelSetup& L0 = H.L[0];
    copy_dev(L0.A.v, vals0, L0.A.nnzb * L0.b * L0.b * sizeof(double), s);
    if (B0) copy_dev(L0.B, B0, L0.A.nr * L0.b * L0.k * sizeof(double), s);
    for (size_t l = 0; l < H.L.size(); ++l) {
        LevelSetup& L = H.L[l];
        level_diag(L, (int)l, err, lamd, s);
        if (l + 1 == H.L.size()) break;
        LevelSetup& N = H.L[l + 1];
        const int64_t nr = L.A.nr, na = L.nagg;
        const int b = L.b, kk = L.k;
        const int64_t g = cdiv(nr, 256);
        // tentative prolongator, coarse near-null space and dead dofs from the kept aggregates
        double* Q = ar.make<double>(nr * b * kk);
        zero_dev(Q, nr * b * kk * sizeof(double), s);
        zero_dev(L.dead, na * kk, s);
        tentative_run(na, b, kk, L.mrp, L.mem, L.B, Q, N.B, L.dead, ar, s);
        DBsr Pt;
        Pt.nr = nr; Pt.nc = na; Pt.br = b; Pt.bc = kk;
        Pt.rp = ar.make<int32_t>(nr + 1);
        int32_t* pc = ar.make<int32_t>(nr + 1);
        ptent_cnt_k<<<g, 256, 0, s>>>(nr, L.agg, pc);
        Pt.nnzb = scan_i32(pc, Pt.rp, nr, ar, s);
        ar.free(pc);
        Pt.ci = ar.make<int32_t>(Pt.nnzb + 1);
        Pt.v = ar.make<double>((Pt.nnzb + 1) * b * kk);
        ptent_fill_k<<<g, 256, 0, s>>>(nr, b * kk, L.agg, Pt.rp, Q, Pt.ci, Pt.v);
        check_launch("ptent");
        // smoothed prolongator into its kept pattern
        spgemm_numeric(L.A, Pt, L.P, ar, s);
        bsr_release(Pt, ar);
        double omega = 4.0 / (3.0 * L.lam);
        if (b == 1 && kk == 1) smooth_p_k<1, 1><<<g, 256, 0, s>>>(nr, L.P.rp, L.P.ci, L.P.v, L.Dinv, L.agg, Q, omega);
        else if (b == 3 && kk == 6) smooth_p_k<3, 6><<<g, 256, 0, s>>>(nr, L.P.rp, L.P.ci, L.P.v, L.Dinv, L.agg, Q, omega);
        else if (b == 6 && kk == 6) smooth_p_k<6, 6><<<g, 256, 0, s>>>(nr, L.P.rp, L.P.ci, L.P.v, L.Dinv, L.agg, Q, omega);
        else throw Error(SCR_E_UNIMPLEMENTED, "prolongator block shape");
        check_launch("smooth_p");
        ar.free(Q);
        bsr_release(L.R, ar);
        L.R = transpose(L.P, ar, s);
        // Galerkin product into the kept patterns of A P and A_{l+1}
        L.AP.v = ar.make<double>((L.AP.nnzb > 0 ? L.AP.nnzb : 1) * L.AP.br * L.AP.bc);
        spgemm_numeric(L.A, L.P, L.AP, ar, s);
        spgemm_numeric(L.R, L.AP, N.A, ar, s);
        ar.free(L.AP.v);
        L.AP.v = nullptr;
        if (na) dead_diag_k<<<cdiv(na, 256), 256, 0, s>>>(na, kk, N.A.rp, N.A.ci, N.A.v, L.dead);
        check_launch("dead_diag");
    }
    coarse_inverse(H, err, ar, s);
    ar.free(err);
    ar.free(lamd);
    H.refresh(ar, s);
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace scr
