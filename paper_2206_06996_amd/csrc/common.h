// common.h -- shared host/device definitions of the gfx950 SCR+AMG library.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/scr.h"

namespace scr {

constexpr int WAVE = 64;       // CDNA wavefront
constexpr int NXCD = 8;        // MI355X: 8 XCDs, workgroups dispatched round-robin

struct Error : std::runtime_error {
    scr_status code;
    Error(scr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& m);

// The status an exception maps to at the C boundary (its message becomes the thread's last error):
// the library's own errors carry their status, a failed host allocation is SCR_E_OOM, anything else
// SCR_E_HIP.
inline scr_status status_of(const std::exception& e) {
    set_last_error(e.what());
    if (const Error* se = dynamic_cast<const Error*>(&e)) return se->code;
    if (dynamic_cast<const std::bad_alloc*>(&e)) return SCR_E_OOM;
    return SCR_E_HIP;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw ::scr::Error(e_ == hipErrorOutOfMemory ? SCR_E_OOM : SCR_E_HIP,                 \
                               std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(SCR_E_HIP, std::string("launch ") + what + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- device memory accounting
// Event-pair timing of one kernel family (opt-in, for the roofline measurement).
struct Profiler {
    std::atomic<int> kernel{0};
    std::mutex mu;
    struct Pending { hipEvent_t a, b; double bytes; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
    hipEvent_t get() {
        std::lock_guard<std::mutex> g(mu);
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(SCR_E_HIP, "hipEventCreate failed");
        }
        return e;
    }
    void push(hipEvent_t a, hipEvent_t b, double by) {
        std::lock_guard<std::mutex> g(mu);
        pending.push_back({a, b, by});
    }
    // fold completed pairs into the totals (callers have synchronised the streams)
    void harvest() {
        std::lock_guard<std::mutex> g(mu);
        std::vector<Pending> keep;
        for (auto& p : pending) {
            float t = 0.f;
            if (hipEventQuery(p.b) != hipSuccess) { keep.push_back(p); continue; }
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) { ms += t; bytes += p.bytes; ++launches; }
            pool.push_back(p.a); pool.push_back(p.b);
        }
        pending.swap(keep);
        (void)hipGetLastError();
    }
};

// Pinned, device-mapped host slots (16 doubles each) through which single-block finishing
// kernels publish Krylov status (residual estimates, flags) with a sequence number the host
// spins on; shared by all handles of a context (handles are created and destroyed per Newton
// corrector, and pinned allocation and release are synchronous and slow).
struct PinnedPool {
    std::mutex mu;
    std::vector<double*> free_;
    std::vector<void*> chunks;
    double* get() {
        std::lock_guard<std::mutex> g(mu);
        if (free_.empty()) {
            void* c = nullptr;
            if (hipHostMalloc(&c, 64 * 16 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
                (void)hipGetLastError();
                throw Error(SCR_E_OOM, "hipHostMalloc of the Krylov status slots failed");
            }
            std::memset(c, 0, 64 * 16 * sizeof(double));
            chunks.push_back(c);
            for (int i = 0; i < 64; ++i) free_.push_back(static_cast<double*>(c) + 16 * i);
        }
        double* p = free_.back();
        free_.pop_back();
        return p;
    }
    // device address of a slot
    static double* device_ptr(double* h) {
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(SCR_E_HIP, "hipHostGetDevicePointer failed");
        }
        return static_cast<double*>(d);
    }
    void put(double* p) {
        std::lock_guard<std::mutex> g(mu);
        free_.push_back(p);
    }
    ~PinnedPool() {
        for (void* c : chunks) (void)hipHostFree(c);
    }
};

// Device blocks released by destroyed handles, kept for the next handles of the context (the
// setup of a new matrix allocates the same sizes again).  Blocks enter only after the stream that
// last used them has been synchronised, so any stream may take them.  Bounded by `cap` bytes.
struct BlockCache {
    std::mutex mu;
    std::multimap<size_t, void*> blocks;
    int64_t bytes = 0;
    int64_t cap = int64_t(16) << 30;
    void* take(size_t n) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = blocks.find(n);
        if (it == blocks.end()) return nullptr;
        void* p = it->second;
        blocks.erase(it);
        bytes -= (int64_t)n;
        return p;
    }
    void put(void* p, size_t n) {
        std::lock_guard<std::mutex> lk(mu);
        blocks.emplace(n, p);
        bytes += (int64_t)n;
        while (bytes > cap && !blocks.empty()) {      // drop the largest blocks first
            auto it = std::prev(blocks.end());
            (void)hipFreeAsync(it->second, nullptr);
            bytes -= (int64_t)it->first;
            blocks.erase(it);
        }
    }
    void flush() {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : blocks) (void)hipFreeAsync(kv.second, nullptr);
        if (!blocks.empty()) (void)hipStreamSynchronize(nullptr);
        blocks.clear();
        bytes = 0;
    }
};

struct Ctx {
    int device = 0;
    int64_t budget = 0;
    std::atomic<int64_t> in_use{0};
    int cu_count = 256;
    Profiler prof;
    PinnedPool pinned;
    BlockCache cache;
};

// Every allocation of a handle goes through an Arena: counted against the context budget and
// released in full when the arena is destroyed.  Sizes are rounded to classes (256 B, then eighths
// of a power of two) so that freed blocks can serve later requests: a block freed during the
// arena's life is reused by the same arena (its work is ordered on the same stream); at the end
// every block goes, after a stream synchronisation, to the context's cache.  New memory comes
// from hipMallocAsync only when neither has a block of the class.
class Arena {
   public:
    Arena(Ctx* c, hipStream_t s) : ctx_(c), stream_(s) {}
    ~Arena() { release_all(); }
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;
    void set_stream(hipStream_t s) {
        if (s != stream_ && !spare_.empty()) (void)hipStreamSynchronize(stream_);
        stream_ = s;
    }
    static size_t size_class(size_t bytes) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes <= 65536) return bytes;
        size_t top = size_t(1) << (63 - __builtin_clzll(bytes));
        size_t step = top >> 3;
        return (bytes + step - 1) / step * step;
    }
    void* alloc(size_t req) {
        size_t bytes = size_class(req);
        if (ctx_->budget > 0 && ctx_->in_use.load() + (int64_t)bytes > ctx_->budget)
            throw Error(SCR_E_OOM, "device memory budget exceeded");
        void* p = nullptr;
        auto it = spare_.find(bytes);
        if (it != spare_.end()) {
            p = it->second;
            spare_.erase(it);
        }
        if (!p) p = ctx_->cache.take(bytes);
        if (!p) {
            hipError_t e = hipMallocAsync(&p, bytes, stream_);
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                ctx_->cache.flush();
                p = nullptr;
                e = hipMallocAsync(&p, bytes, stream_);
                if (e != hipSuccess || !p) {
                    (void)hipGetLastError();
                    throw Error(SCR_E_OOM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
                }
            }
        }
        ctx_->in_use += (int64_t)bytes;
        bytes_ += (int64_t)bytes;
        if (bytes_ > peak_) peak_ = bytes_;
        live_.push_back({p, bytes});
        return p;
    }
    template <typename T>
    T* make(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
    void free(void* p) {
        if (!p) return;
        for (size_t i = 0; i < live_.size(); ++i)
            if (live_[i].p == p) {
                spare_.emplace(live_[i].n, p);
                ctx_->in_use -= (int64_t)live_[i].n;
                bytes_ -= (int64_t)live_[i].n;
                live_[i] = live_.back();
                live_.pop_back();
                return;
            }
    }
    void release_all() {
        if (live_.empty() && spare_.empty()) return;
        (void)hipStreamSynchronize(stream_);
        for (auto& a : live_) {
            ctx_->cache.put(a.p, a.n);
            ctx_->in_use -= (int64_t)a.n;
        }
        for (auto& kv : spare_) ctx_->cache.put(kv.second, kv.first);
        live_.clear();
        spare_.clear();
        bytes_ = 0;
    }
    int64_t bytes() const { return bytes_; }
    int64_t peak() const { return peak_; }
    hipStream_t stream() const { return stream_; }
    Ctx* ctx() const { return ctx_; }

   private:
    struct A { void* p; size_t n; };
    Ctx* ctx_;
    hipStream_t stream_;
    std::vector<A> live_;
    std::multimap<size_t, void*> spare_;
    int64_t bytes_ = 0;
    int64_t peak_ = 0;     // largest bytes_ ever held
};

// ---------------------------------------------------------------- matrices
// Block CSR on the device, FP64 values (setup form, and the form inspected by tests).
struct DBsr {
    int64_t nr = 0, nc = 0;
    int br = 0, bc = 0;
    int64_t nnzb = 0;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* v = nullptr;
};

// Sliced ELL, two lane mappings.
//
// Scalar-row lanes (every shape but 3x3 and 3x6).  A slice is one wavefront covering rps = 64/br block
// rows (lanes = rps*br; the rest idle), so the br lanes of a block row share a wavefront.  Lane
// (block row i, row r) reads, for every slot t of the slice, the column block index of block row
// i (stored once per block row) and row r of that block (bc values); each of the bc entries of a
// slot is a 64-wide contiguous vector, so every load is fully coalesced and no cross-lane sum
// is needed.
//   col of (slice s, slot t, block row j of the slice):   ci[(off[s] + t) * rps + j]
//   entry k of lane l's row segment:                       v[((off[s] + t) * bc + k) * 64 + l]
//
// Block-row lanes (3x3 blocks: the velocity block and its FP32 copy; 3x6: the prolongators of
// AMG(A)).  A slice is one wavefront covering rps = 64 block rows, one per lane; the lane computes
// all three rows of its block row.  Each lane gathers the bc-vector of x at its column once (the
// scalar-row mapping gathers it three times, once per row lane), which is what these sweeps are
// bound by.
//   col of (slice s, slot t, lane l):                      ci[(off[s] + t) * 64 + l]
//   entry e = bc*r + k of the block at (s, t, l):          v[((off[s] + t) * 3*bc + e) * 64 + l]
//
// Rows shorter than the slice are padded with zero entries pointing at a valid column.  Within
// windows of sigma slices, block rows are ordered by decreasing length (ties by index) so that
// rows of similar length share a slice; rowid maps slice positions back to block rows (-1 =
// empty position).  sigma trades padding against the spread of the gathered x entries: 16
// slices of 21 rows for scalar-row lanes, 6 slices of 64 rows for block-row lanes (measured).
constexpr int SELL_SIGMA = 16;
constexpr int SELL_SIGMA_ROWLANE = 6;
template <typename T>
struct DSell {
    int64_t nr = 0, nc = 0;
    int br = 0, bc = 0;
    int rps = 0;                // block rows per slice
    bool rowlane = false;       // block-row lanes (3x3) instead of scalar-row lanes
    int64_t nslices = 0;
    int64_t slots = 0;          // sum over slices of the slice length
    int64_t nnzb = 0;           // stored blocks before padding (algorithmic count)
    int32_t* off = nullptr;     // nslices + 1 (slot offsets)
    int32_t* rowid = nullptr;   // nslices * rps
    int32_t* ci = nullptr;
    T* v = nullptr;
};

// ---------------------------------------------------------------- launch helpers
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Map the hardware workgroup id to a logical tile so that each XCD (its own L2) receives one
// contiguous range of tiles: neighbouring rows share the gathered x entries through that L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    int64_t q = nb / NXCD, r = nb % NXCD;
    int64_t x = b % NXCD, k = b / NXCD;
    return x * q + (x < r ? x : r) + k;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

}  // namespace scr

// The opaque context of the C ABI.
struct scr_ctx {
    scr::Ctx c;
};
