// common.h -- shared host/device definitions of the gfx950 SCR+AMG library.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
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
struct Ctx {
    int device = 0;
    int64_t budget = 0;
    std::atomic<int64_t> in_use{0};
    int cu_count = 256;
};

// Every allocation of a handle goes through an Arena: stream-ordered, counted against the
// context budget, and released in full when the arena is destroyed.
class Arena {
   public:
    Arena(Ctx* c, hipStream_t s) : ctx_(c), stream_(s) {}
    ~Arena() { release_all(); }
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;
    void set_stream(hipStream_t s) { stream_ = s; }
    void* alloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        if (ctx_->budget > 0 && ctx_->in_use.load() + (int64_t)bytes > ctx_->budget)
            throw Error(SCR_E_OOM, "device memory budget exceeded");
        void* p = nullptr;
        hipError_t e = hipMallocAsync(&p, bytes, stream_);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw Error(SCR_E_OOM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
        }
        ctx_->in_use += (int64_t)bytes;
        bytes_ += (int64_t)bytes;
        live_.push_back({p, bytes});
        return p;
    }
    template <typename T>
    T* make(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
    void free(void* p) {
        if (!p) return;
        for (size_t i = 0; i < live_.size(); ++i)
            if (live_[i].p == p) {
                (void)hipFreeAsync(p, stream_);
                ctx_->in_use -= (int64_t)live_[i].n;
                bytes_ -= (int64_t)live_[i].n;
                live_[i] = live_.back();
                live_.pop_back();
                return;
            }
    }
    void release_all() {
        for (auto& a : live_) {
            (void)hipFreeAsync(a.p, stream_);
            ctx_->in_use -= (int64_t)a.n;
        }
        live_.clear();
        bytes_ = 0;
    }
    int64_t bytes() const { return bytes_; }
    hipStream_t stream() const { return stream_; }

   private:
    struct A { void* p; size_t n; };
    Ctx* ctx_;
    hipStream_t stream_;
    std::vector<A> live_;
    int64_t bytes_ = 0;
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

// Sliced ELL with 64-row slices (one wavefront per slice, one lane per block row).  Within a
// slice, slot t of every row is stored lane-contiguously, and each block entry e of that slot
// is a 64-wide contiguous vector: loads are fully coalesced and need no cross-lane reduction.
//   col of (slice s, slot t, lane l):   ci[(off[s] + t) * 64 + l]
//   entry e of that block:              v[((off[s] + t) * br*bc + e) * 64 + l]
// Short rows are padded with zero blocks whose column is a valid index.
template <typename T>
struct DSell {
    int64_t nr = 0, nc = 0;
    int br = 0, bc = 0;
    int64_t nslices = 0;
    int64_t slots = 0;          // sum over slices of the slice length
    int64_t nnzb = 0;           // stored blocks before padding (algorithmic count)
    int32_t* off = nullptr;     // nslices + 1 (slot offsets)
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
