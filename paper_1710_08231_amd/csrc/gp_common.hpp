// gp_common.hpp — internal definitions shared by the gfx950 kernels of the
// label-propagation partitioner: error plumbing, the per-call scratch
// allocator (stream-ordered), and wave64 / workgroup primitives.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "gp.h"

namespace gp {

constexpr int kWave = 64;

void set_error(const char *msg);
const char *last_error();

// Host time spent in stream-ordered allocation calls (reported by GP_TRACE=1).
struct AllocStats {
    double host_ms = 0;
    int64_t calls = 0, bytes = 0;
};
AllocStats &alloc_stats();

// GP_TRACE=2: every scratch request is printed to stderr (size, bytes held after it).
inline bool trace_allocs() {
    static const bool on = [] {
        const char *e = std::getenv("GP_TRACE");
        return e && e[0] == '2';
    }();
    return on;
}

inline hipError_t timed_malloc_async(void **p, size_t bytes, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const hipError_t e = hipMallocAsync(p, bytes, s);
    AllocStats &a = alloc_stats();
    a.host_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    a.calls++;
    a.bytes += (int64_t)bytes;
    return e;
}

// Returns GP_ERR_HIP (with a message) when a HIP call fails.
#define GP_HIP(expr)                                                              \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) {                                                   \
            ::gp::set_error((std::string(#expr) + ": " + hipGetErrorString(_e)).c_str()); \
            return GP_ERR_HIP;                                                    \
        }                                                                         \
    } while (0)

#define GP_TRY(expr)                  \
    do {                              \
        int _rc = (expr);             \
        if (_rc < 0) return _rc;      \
    } while (0)

#define GP_LAUNCH_CHECK() GP_HIP(hipGetLastError())

// Per-(device, stream) cache of device memory reused by successive library
// calls on that stream: a list of large blocks served as a bump allocator by
// one call at a time and rewound when the call ends. Work is ordered on the
// stream, so a later call may reuse the memory of an earlier one at once.
// Blocks are allocated stream-ordered and kept until gp_release_cache().
struct Arena {
    struct Block {
        char *p;
        size_t size;
    };
    std::vector<Block> blocks;
    size_t cur = 0, off = 0;
    size_t used = 0;    // bytes the current call holds (less what it rewound)
    size_t need = 0;    // the current call's high-water mark of `used`
    bool grew = false;  // the current call had to add a block
    bool busy = false;
};
// The arena of (current device, s), created on first use; null on failure.
Arena *arena_for(hipStream_t s);

// Scratch memory for one library call. Three sources:
//  - the stream's arena (or, if that arena is already serving another live
//    Scratch, hipMallocAsync blocks freed on release);
//  - caller memory [ws, ws + ws_bytes): carved as a bump allocator, nothing is
//    ever allocated, and a request that does not fit fails with
//    GP_ERR_WORKSPACE;
//  - the same, for a buffer the library owns statically (set_static()): the
//    call then also creates no HIP events, streams or graphs.
// Everything is given back when the object goes out of scope.
class Scratch {
  public:
    explicit Scratch(hipStream_t s) : s_(s) { use_cache(); }
    Scratch(hipStream_t s, void *ws, size_t ws_bytes) : s_(s) {
        if (!ws) {
            use_cache();
            return;
        }
        fixed_ = true;
        const uintptr_t b = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
        const size_t lost = (size_t)(b - (uintptr_t)ws);
        own_.blocks.push_back({reinterpret_cast<char *>(b), ws_bytes > lost ? ws_bytes - lost : 0});
        own_.busy = true;
        a_ = &own_;
    }
    // the buffer is the library's own static scratch: no runtime objects either
    void set_static() { static_ = true; }
    bool is_static() const { return static_; }
    bool fixed() const { return fixed_; }
    ~Scratch() { release(); }
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;

    template <typename T>
    int alloc(T **out, size_t count) {
        void *p = nullptr;
        const size_t bytes = ((count ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
        if (a_) {
            const int rc = take(bytes, &p);
            *out = static_cast<T *>(p);
            return rc;
        }
        hipError_t e = timed_malloc_async(&p, bytes, s_);
        if (e != hipSuccess) {
            set_error((std::string("hipMallocAsync(") + std::to_string(bytes) + "): " +
                       hipGetErrorString(e)).c_str());
            *out = nullptr;
            return GP_ERR_HIP;
        }
        ptrs_.push_back(p);
        *out = static_cast<T *>(p);
        return GP_OK;
    }
    // Reusable buffer `slot` of at least `count` elements, kept for the life of
    // this object. Work is stream ordered, so successive users of one slot
    // never overlap.
    template <typename T>
    int temp(T **out, size_t count, int slot) {
        const size_t bytes = (count ? count : 1) * sizeof(T);
        if (slot >= (int)tmp_.size()) {
            if (frozen_) return frozen_fail();
            tmp_.resize(slot + 1, {nullptr, 0});
        }
        if (tmp_[slot].second < bytes) {
            if (frozen_) return frozen_fail();
            const size_t grow = bytes + bytes / 4;
            char *p = nullptr;
            GP_TRY(alloc(&p, grow));  // the outgrown buffer returns with the rest at release
            tmp_[slot] = {p, grow};
        }
        *out = static_cast<T *>(tmp_[slot].first);
        return GP_OK;
    }
    // A point to come back to: everything taken after mark() is given back to
    // this call's arena by rewind(mark), so later allocations of the same call
    // reuse it (work is stream ordered). Reusable slots grown after the mark
    // return to their earlier buffers.
    struct Mark {
        size_t cur = 0, off = 0, used = 0;
        bool arena = false;
        std::vector<std::pair<void *, size_t>> tmp;
    };
    Mark mark() const {
        Mark m;
        m.tmp = tmp_;
        if (a_) {
            m.arena = true;
            m.cur = a_->cur;
            m.off = a_->off;
            m.used = a_->used;
        }
        return m;
    }
    void rewind(const Mark &m) {
        if (!a_ || !m.arena) return;
        a_->cur = m.cur;
        a_->off = m.off;
        a_->used = m.used;
        tmp_ = m.tmp;
    }
    void release() {
        for (void *p : ptrs_) (void)hipFreeAsync(p, s_);
        ptrs_.clear();
        tmp_.clear();
        if (a_) {
            if (!fixed_ && a_->grew && a_->blocks.size() > 1) consolidate();
            if (fixed_) need_fixed_ = a_->need;
            a_->cur = 0;
            a_->off = 0;
            a_->used = 0;
            a_->need = 0;
            a_->grew = false;
            a_->busy = false;
            a_ = nullptr;
        }
    }
    // bytes of scratch this call has held at once so far (0 without a cache)
    size_t high_water() const { return a_ ? a_->need : (fixed_ ? need_fixed_ : 0); }
    hipStream_t stream() const { return launch_ ? launch_ : s_; }
    // Launch subsequent work on `st` (for recording a launch sequence); while
    // `frozen`, scratch slots may not grow, so nothing is allocated.
    void set_stream(hipStream_t st, bool frozen) {
        launch_ = st == s_ ? nullptr : st;
        frozen_ = frozen;
    }

  private:
    void use_cache() {
        keep_pool();
        a_ = arena_for(s_);
        if (a_ && !a_->busy) {
            a_->busy = true;
            a_->cur = 0;
            a_->off = 0;
            a_->used = 0;
            a_->need = 0;
        } else {
            a_ = nullptr;
        }
    }
    static constexpr size_t kMinBlock = size_t(512) << 20;
    // After a call that had to grow the cache, replace its blocks by one block
    // of the call's high-water mark plus 1/16, so a call with the same needs
    // fits without gaps (also when its needs vary by a little: growing again
    // means freeing, trimming and mapping the whole cache anew, seconds of host
    // time for tens of GB) and the cache does not accumulate blocks.
    void consolidate() {
        for (auto &b : a_->blocks) (void)hipFreeAsync(b.p, s_);
        a_->blocks.clear();
        (void)hipStreamSynchronize(s_);
        int dev = 0;
        hipMemPool_t pool;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
            (void)hipMemPoolTrimTo(pool, 0);
        void *q = nullptr;
        const size_t size = a_->need + a_->need / 16;
        if (timed_malloc_async(&q, size, s_) == hipSuccess) a_->blocks.push_back({static_cast<char *>(q), size});
        else (void)hipGetLastError();  // the next call grows the cache again
    }
    int take(size_t bytes, void **p) {
        a_->used += bytes;
        if (a_->used > a_->need) a_->need = a_->used;
        if (trace_allocs()) std::fprintf(stderr, "[gp alloc] %zu used %zu\n", bytes, a_->used);
        while (a_->cur < a_->blocks.size()) {
            Arena::Block &b = a_->blocks[a_->cur];
            if (a_->off + bytes <= b.size) {
                *p = b.p + a_->off;
                a_->off += bytes;
                return GP_OK;
            }
            if (fixed_) break;
            a_->cur++;
            a_->off = 0;
        }
        if (fixed_) {
            set_error((std::string("workspace too small: the call needs more than ") + std::to_string(a_->used) +
                       " bytes of scratch at once, the workspace holds " + std::to_string(a_->blocks[0].size) +
                       " (after aligning it to 256 bytes)").c_str());
            *p = nullptr;
            return GP_ERR_WORKSPACE;
        }
        void *q = nullptr;
        const size_t size = bytes > kMinBlock ? bytes : kMinBlock;
        hipError_t e = timed_malloc_async(&q, size, s_);
        if (e != hipSuccess) {
            set_error((std::string("hipMallocAsync(") + std::to_string(size) + "): " + hipGetErrorString(e)).c_str());
            *p = nullptr;
            return GP_ERR_HIP;
        }
        a_->blocks.push_back({static_cast<char *>(q), size});
        a_->grew = true;
        a_->cur = a_->blocks.size() - 1;
        a_->off = bytes;
        *p = q;
        return GP_OK;
    }
    int frozen_fail() {
        set_error("scratch slot would grow while a launch sequence is recorded");
        return GP_ERR_HIP;
    }
    // Keep freed blocks in the device's default pool instead of returning them
    // to the driver at every synchronisation.
    static void keep_pool() {
        static bool done = false;
        if (done) return;
        int dev = 0;
        hipMemPool_t pool;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        done = true;
    }
    hipStream_t s_;
    hipStream_t launch_ = nullptr;
    bool frozen_ = false;
    bool fixed_ = false, static_ = false;
    size_t need_fixed_ = 0;
    Arena own_;  // the single block of caller (or static) memory
    Arena *a_ = nullptr;
    std::vector<void *> ptrs_;
    std::vector<std::pair<void *, size_t>> tmp_;
};

// Gives back, when it goes out of scope, everything its Scratch handed out
// since the scope began (for calls whose scratch is all internal: results in
// caller buffers or on the host).
struct ScratchScope {
    Scratch &sc;
    Scratch::Mark m;
    explicit ScratchScope(Scratch &s) : sc(s), m(s.mark()) {}
    ~ScratchScope() { sc.rewind(m); }
    ScratchScope(const ScratchScope &) = delete;
    ScratchScope &operator=(const ScratchScope &) = delete;
};

// ---------------------------------------------------------------- instrumentation
// When enabled (gp_profile_enable), selected kernel launches are bracketed by
// HIP events on their stream; durations and the algorithmic bytes of each
// launch accumulate per kernel name (optionally prefixed by the phase and
// level set with prof_context) until read back (gp_profile_get).
bool prof_on();
bool prof_wants(const char *name);
// true when every launch is to be bracketed, so rounds must not be replayed
bool prof_blocks_replay();
// LP-call events (whole gp clustering / refinement runs per level)
bool prof_calls();
// while suspended no event is recorded (a launch sequence recorded for
// replay; the rounds after the first under GP_PROFILE_EAGER)
void prof_suspend(bool on);
// GP_PROFILE_EAGER without GP_PROFILE_KERNELS: only the first round of every
// LP run is sampled, so the rounds that follow run without events
bool prof_first_round_only();
struct ProfSuspend {
    bool on;
    explicit ProfSuspend(bool b) : on(b) {
        if (on) prof_suspend(true);
    }
    ~ProfSuspend() {
        if (on) prof_suspend(false);
    }
};
void prof_context(const char *ctx);
void prof_record(const char *name, hipEvent_t a, hipEvent_t b, double bytes);
hipEvent_t prof_event();
void prof_flush();  // resolves recorded events (the stream must be synchronised)

#define GP_PROF_LAUNCH(name, bytes, stream, ...)                     \
    do {                                                              \
        if (::gp::prof_wants(name)) {                                 \
            hipEvent_t _a = ::gp::prof_event(), _b = ::gp::prof_event(); \
            (void)hipEventRecord(_a, stream);                         \
            __VA_ARGS__;                                              \
            (void)hipEventRecord(_b, stream);                         \
            ::gp::prof_record(name, _a, _b, (double)(bytes));         \
        } else {                                                      \
            __VA_ARGS__;                                              \
        }                                                             \
    } while (0)

inline unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

inline int bits_for(int64_t maxval) {  // bits needed to represent values in [0, maxval]
    int b = 0;
    while (b < 63 && (int64_t(1) << b) <= maxval) b++;
    return b;
}

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// a[key] += x over the lanes with `valid`: one atomic for the wave when all of
// them share one key (entries grouped by graph or label), else one per lane.
// Every lane of the wave calls it.
template <typename T>
__device__ __forceinline__ void wave_add_keyed(T *a, int32_t key, T x, bool valid) {
    const uint64_t vm = __ballot(valid);
    if (!vm) return;
    const int32_t k0 = __shfl(key, __ffsll((unsigned long long)vm) - 1, kWave);
    if (__ballot(valid && key != k0) == 0) {
        T v = valid ? x : T(0);
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
        if (lane_id() == 0) atomicAdd(&a[k0], v);
    } else if (valid) {
        atomicAdd(&a[key], x);
    }
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        T y = __shfl_xor(x, d, kWave);
        x = y > x ? y : x;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        T y = __shfl_xor(x, d, kWave);
        x = y < x ? y : x;
    }
    return x;
}

// Workgroup-wide exclusive scan; `tmp` must hold BLOCK/64 + 1 elements.
// Returns the thread's exclusive prefix; *total receives the block sum.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *tmp, T *total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    T inc = wave_incl_scan(x);
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < NW; i++) {
            T t = tmp[i];
            tmp[i] = acc;
            acc += t;
        }
        tmp[NW] = acc;
    }
    __syncthreads();
    T r = tmp[w] + inc - x;
    if (total) *total = tmp[NW];
    __syncthreads();
    return r;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T x, T *tmp) {
    constexpr int NW = BLOCK / kWave;
    T s = wave_sum(x);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) tmp[w] = s;
    __syncthreads();
    T r = 0;
    for (int i = 0; i < NW; i++) r += tmp[i];
    __syncthreads();
    return r;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_min(T x, T *tmp) {
    constexpr int NW = BLOCK / kWave;
    T s = wave_min(x);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) tmp[w] = s;
    __syncthreads();
    T r = tmp[0];
    for (int i = 1; i < NW; i++) r = tmp[i] < r ? tmp[i] : r;
    __syncthreads();
    return r;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_max(T x, T *tmp) {
    constexpr int NW = BLOCK / kWave;
    T s = wave_max(x);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) tmp[w] = s;
    __syncthreads();
    T r = tmp[0];
    for (int i = 1; i < NW; i++) r = tmp[i] > r ? tmp[i] : r;
    __syncthreads();
    return r;
}

// 8 XCDs: consecutive block ids are dealt round-robin to XCDs. Remap so each
// XCD works on one contiguous range of tiles (shared L2 lines between
// neighbouring CSR rows stay in one L2).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks) {
    constexpr unsigned X = 8;
    if (nblocks < X || (nblocks % X) != 0) return b;
    return (b % X) * (nblocks / X) + b / X;
}

}  // namespace gp
