// prims.hpp — device-wide building blocks for gfx950: reduce-then-scan prefix
// sums with fused input/output functors (scan, stable compaction, segmented
// scans), and a stable LSD radix sort with 8-bit digits.
//
// Item counts may live on the device (`n_dev`): grids are sized for `nmax`
// and tiles past the live count do nothing, so no host round trip is needed.
#pragma once
#include "gp_common.hpp"

namespace gp {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ int64_t live_count(int64_t nmax, const int32_t *n_dev) {
    if (!n_dev) return nmax;
    int64_t n = *n_dev;
    return n < nmax ? n : nmax;
}

// ---------------------------------------------------------------- scan

template <typename T, typename In>
__global__ __launch_bounds__(kScanBlock) void k_tile_reduce(In in, int64_t nmax, const int32_t *n_dev,
                                                            T *partial) {
    __shared__ T tmp[kScanBlock / kWave + 1];
    const int64_t n = live_count(nmax, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
    if (base < n) {
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            int64_t idx = base + (int64_t)i * kScanBlock + threadIdx.x;
            if (idx < n) s += in(idx);
        }
    }
    s = block_sum<kScanBlock>(s, tmp);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Each thread owns kScanItems consecutive items (blocked layout) so the
// output functor sees items in ascending order within the thread.
template <typename T, typename In, typename Out>
__global__ __launch_bounds__(kScanBlock) void k_tile_scan(In in, Out out, int64_t nmax,
                                                          const int32_t *n_dev, const T *tile_off,
                                                          T *total) {
    __shared__ T tmp[kScanBlock / kWave + 1];
    const int64_t n = live_count(nmax, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    if (base >= n && !(blockIdx.x == 0 && total)) return;
    T v[kScanItems];
    T s = 0;
    const int64_t mine = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        int64_t idx = mine + i;
        v[i] = idx < n ? in(idx) : T(0);
        s += v[i];
    }
    T tot;
    T ex = block_excl_scan<kScanBlock>(s, tmp, &tot);
    T off = tile_off ? tile_off[blockIdx.x] : T(0);
    ex += off;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        int64_t idx = mine + i;
        if (idx < n) out(idx, ex, v[i]);
        ex += v[i];
    }
    if (total && threadIdx.x == 0) {
        const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
        if (n == 0 && blockIdx.x == 0) *total = 0;
        else if ((int64_t)blockIdx.x == ntiles - 1) *total = off + tot;
    }
}

template <typename T>
struct LoadIn {
    const T *p;
    __device__ T operator()(int64_t i) const { return p[i]; }
};
template <typename T>
struct StoreExcl {
    T *p;
    __device__ void operator()(int64_t i, T ex, T) const { p[i] = ex; }
};

// Exclusive scan of in(i), i < n (n = min(nmax, *n_dev) when n_dev is set);
// out(i, exclusive_prefix, value) is called once per item; *total_dev (may be
// NULL) receives the sum.
template <typename T, typename In, typename Out>
int scan(In in, Out out, int64_t nmax, const int32_t *n_dev, T *total_dev, Scratch &sc, int depth = 0) {
    hipStream_t s = sc.stream();
    const int64_t ntiles = (nmax + kScanTile - 1) / kScanTile;
    if (ntiles <= 1) {
        hipLaunchKernelGGL((k_tile_scan<T, In, Out>), dim3(1), dim3(kScanBlock), 0, s, in, out, nmax,
                           n_dev, (const T *)nullptr, total_dev);
        GP_LAUNCH_CHECK();
        return GP_OK;
    }
    T *partial = nullptr, *off = nullptr;
    GP_TRY(sc.temp(&partial, ntiles, 2 * depth));
    GP_TRY(sc.temp(&off, ntiles, 2 * depth + 1));
    hipLaunchKernelGGL((k_tile_reduce<T, In>), dim3(ntiles), dim3(kScanBlock), 0, s, in, nmax, n_dev,
                       partial);
    GP_LAUNCH_CHECK();
    GP_TRY((scan<T>(LoadIn<T>{partial}, StoreExcl<T>{off}, ntiles, nullptr, (T *)nullptr, sc, depth + 1)));
    hipLaunchKernelGGL((k_tile_scan<T, In, Out>), dim3(ntiles), dim3(kScanBlock), 0, s, in, out, nmax,
                       n_dev, (const T *)off, total_dev);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

struct DiscardOut {
    template <typename T>
    __device__ void operator()(int64_t, T, T) const {}
};

// Sum of in(i), i < n, into *total_dev: one pass of tile sums, then the same
// over the tile sums until one tile is left.
template <typename T, typename In>
int reduce(In in, int64_t nmax, const int32_t *n_dev, T *total_dev, Scratch &sc, int depth = 0) {
    hipStream_t s = sc.stream();
    const int64_t ntiles = (nmax + kScanTile - 1) / kScanTile;
    if (ntiles <= 1) {
        hipLaunchKernelGGL((k_tile_scan<T, In, DiscardOut>), dim3(1), dim3(kScanBlock), 0, s, in, DiscardOut{}, nmax,
                           n_dev, (const T *)nullptr, total_dev);
        GP_LAUNCH_CHECK();
        return GP_OK;
    }
    T *partial = nullptr;
    GP_TRY(sc.temp(&partial, ntiles, 2 * depth));
    hipLaunchKernelGGL((k_tile_reduce<T, In>), dim3(ntiles), dim3(kScanBlock), 0, s, in, nmax, n_dev, partial);
    GP_LAUNCH_CHECK();
    return reduce<T>(LoadIn<T>{partial}, ntiles, nullptr, total_dev, sc, depth + 1);
}

// Stable compaction: writes idx-th kept item's index mapping through `emit`.
template <typename Flag, typename Emit>
struct CompactOut {
    Flag flag;
    Emit emit;
    __device__ void operator()(int64_t i, int32_t ex, int32_t v) const {
        if (v) emit(i, ex);
    }
};
template <typename Flag>
struct FlagIn {
    Flag flag;
    __device__ int32_t operator()(int64_t i) const { return flag(i) ? 1 : 0; }
};

template <typename Flag, typename Emit>
int compact(Flag flag, Emit emit, int64_t nmax, const int32_t *n_dev, int32_t *count_dev,
            Scratch &sc) {
    return scan<int32_t>(FlagIn<Flag>{flag}, CompactOut<Flag, Emit>{flag, emit}, nmax, n_dev,
                         count_dev, sc);
}

// ---------------------------------------------------------------- radix sort

constexpr int kSortHistSlot = 16;  // scratch slots 0..15 belong to scan depths
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;

template <typename K>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const K *keys, int64_t nmax,
                                                           const int32_t *n_dev, int shift,
                                                           uint32_t mask, uint32_t *hist,
                                                           int ntiles) {
    __shared__ uint32_t h[256];
    const int64_t n = live_count(nmax, n_dev);
    for (int d = threadIdx.x; d < 256; d += kSortBlock) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int i = 0; i < kSortItems; i++) {
        int64_t idx = base + (int64_t)i * kSortBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kSortBlock) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// Stable scatter of one tile. Each wave owns a contiguous quarter of the
// tile and ranks its items round by round (64 at a time, peers of a digit
// found by ballots over the digit bits) against wave-private digit counters,
// so ranks follow the original order. The tile is then placed in LDS in
// digit order and written out from there: consecutive threads write
// consecutive positions of each digit's run.
template <typename K, typename V>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const K *kin, const V *vin, K *kout,
                                                              V *vout, int64_t nmax,
                                                              const int32_t *n_dev, int shift,
                                                              int nbits, const uint32_t *offs,
                                                              int ntiles) {
    static_assert(kSortBlock == 256, "one thread per digit");
    constexpr int NW = kSortBlock / kWave;
    constexpr int PER_W = kSortTile / NW;
    constexpr int R = PER_W / kWave;
    __shared__ uint32_t wc[NW][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t tmp[NW + 1];
    // the tile passes through LDS twice, keys then values, in one buffer
    constexpr size_t kItem = sizeof(K) > sizeof(V) ? sizeof(K) : sizeof(V);
    __shared__ __align__(16) unsigned char stage[kSortTile * kItem];
    K *sk = reinterpret_cast<K *>(stage);
    V *sv = reinterpret_cast<V *>(stage);
    const int64_t n = live_count(nmax, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    if (base >= n) return;
    const uint32_t mask = (1u << nbits) - 1u;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
    for (int d = threadIdx.x; d < NW * 256; d += kSortBlock) (&wc[0][0])[d] = 0;
    if (offs) goff[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    __syncthreads();
    const int64_t wbase = base + (int64_t)w * PER_W;
    K key[R];
    V val[R];
    uint32_t rk[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int64_t idx = wbase + r * kWave + lane;
        key[r] = idx < n ? kin[idx] : K(0);
        val[r] = idx < n ? vin[idx] : V(0);
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const bool valid = wbase + r * kWave + lane < n;
        const uint32_t dig = (uint32_t)(key[r] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int bt = 0; bt < nbits; bt++) {
            const bool bit = (dig >> bt) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = valid ? wc[w][dig] : 0u;
        const uint32_t pr = (uint32_t)__popcll(peers & lt);
        rk[r] = before + pr;
        // every lane has read the counter before the group's first lane
        // advances it (one wave: LDS operations complete in program order)
        if (valid && pr == 0) wc[w][dig] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t acc = 0;
    for (int q = 0; q < NW; q++) {
        const uint32_t t = wc[q][threadIdx.x];
        wc[q][threadIdx.x] = acc;
        acc += t;
    }
    dstart[threadIdx.x] = block_excl_scan<kSortBlock>(acc, tmp, (uint32_t *)nullptr);
    // one tile alone (offs == null): its own digit starts are the global ones
    if (!offs) goff[threadIdx.x] = dstart[threadIdx.x];
    __syncthreads();
    // local position of each item; its digit is kept for the value pass
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t dig = (uint32_t)(key[r] >> shift) & mask;
        rk[r] += dstart[dig] + wc[w][dig];
        if (wbase + r * kWave + lane < n) sk[rk[r]] = key[r];
    }
    __syncthreads();
    const int32_t cnt = (int32_t)((n - base) < kSortTile ? (n - base) : kSortTile);
    uint8_t pd[kSortTile / kSortBlock];  // digit of each output slot of this thread
#pragma unroll
    for (int q = 0; q < kSortTile / kSortBlock; q++) {
        const int32_t p = threadIdx.x + q * kSortBlock;
        if (p < cnt) {
            const K kk = sk[p];
            const uint32_t dig = (uint32_t)(kk >> shift) & mask;
            pd[q] = (uint8_t)dig;
            kout[goff[dig] + ((uint32_t)p - dstart[dig])] = kk;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++)
        if (wbase + r * kWave + lane < n) sv[rk[r]] = val[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortTile / kSortBlock; q++) {
        const int32_t p = threadIdx.x + q * kSortBlock;
        if (p < cnt) vout[goff[pd[q]] + ((uint32_t)p - dstart[pd[q]])] = sv[p];
    }
}

// Stable LSD sort of (keys, vals) on the low `bits` bits of the key. The
// result is in (*keys, *vals) on return; the pointers may be swapped with the
// temporaries.
template <typename K, typename V>
int radix_sort(K **keys, V **vals, K **ktmp, V **vtmp, int64_t nmax, const int32_t *n_dev, int bits,
               Scratch &sc) {
    hipStream_t s = sc.stream();
    if (nmax <= 0 || bits <= 0) return GP_OK;
    const int ntiles = (int)((nmax + kSortTile - 1) / kSortTile);
    if (ntiles == 1) {  // one tile: one launch per pass ranks, places and writes it
        for (int shift = 0; shift < bits; shift += 8) {
            const int nb = (bits - shift) < 8 ? (bits - shift) : 8;
            hipLaunchKernelGGL((k_radix_scatter<K, V>), dim3(1), dim3(kSortBlock), 0, s, *keys, *vals, *ktmp, *vtmp,
                               nmax, n_dev, shift, nb, (const uint32_t *)nullptr, 1);
            GP_LAUNCH_CHECK();
            K *tk = *keys;
            *keys = *ktmp;
            *ktmp = tk;
            V *tv = *vals;
            *vals = *vtmp;
            *vtmp = tv;
        }
        return GP_OK;
    }
    uint32_t *hist = nullptr;
    GP_TRY(sc.temp(&hist, (size_t)256 * ntiles, kSortHistSlot));
    for (int shift = 0; shift < bits; shift += 8) {
        const int nb = (bits - shift) < 8 ? (bits - shift) : 8;
        hipLaunchKernelGGL((k_radix_hist<K>), dim3(ntiles), dim3(kSortBlock), 0, s, *keys, nmax, n_dev,
                           shift, (1u << nb) - 1u, hist, ntiles);
        GP_LAUNCH_CHECK();
        GP_TRY((scan<uint32_t>(LoadIn<uint32_t>{hist}, StoreExcl<uint32_t>{hist}, (int64_t)256 * ntiles,
                               nullptr, (uint32_t *)nullptr, sc)));
        hipLaunchKernelGGL((k_radix_scatter<K, V>), dim3(ntiles), dim3(kSortBlock), 0, s, *keys, *vals,
                           *ktmp, *vtmp, nmax, n_dev, shift, nb, hist, ntiles);
        GP_LAUNCH_CHECK();
        K *tk = *keys;
        *keys = *ktmp;
        *ktmp = tk;
        V *tv = *vals;
        *vals = *vtmp;
        *vtmp = tv;
    }
    return GP_OK;
}

// ---------------------------------------------------------------- misc kernels

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
int fill(T *p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return GP_OK;
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, p, n, v);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

}  // namespace gp
