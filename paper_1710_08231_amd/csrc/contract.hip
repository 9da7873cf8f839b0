// contract.hip — contraction (§III-A quotient graph; §IV-A relabelling by a
// prefix sum over used labels), projection (§III-C) and the cut (§II-A).
//
// Contraction groups the fine vertices by coarse id instead of the paper's
// concurrent hash table over all cut edges:
//   used[L] flags -> exclusive scan -> f2c[v] = id[C[v]], n'; c'(i) by integer
//   atomics; members of each coarse vertex (counting sort by f2c) and the
//   prefix of their degrees, so coarse row i owns the flattened entry range
//   [flat[mstart[i]], flat[mstart[i+1]]) of length D_i;
//   row i's entries (j = f2c[u], w) with j != i are summed in a hash table
//   keyed by j — in LDS for D_i <= 2048 (one wave per row up to 128 entries,
//   one workgroup per row above), then the distinct columns are sorted in LDS;
//   rows above 2048 entries are inserted chunk-wise into per-row global
//   tables and only their distinct (row, column) pairs are radix sorted;
//   a scan of the per-row column counts gives the coarse row offsets and a
//   copy compacts the rows.
#include <algorithm>
#include <climits>
#include <vector>

#include "contract.hpp"
#include "prims.hpp"

namespace gp {

namespace {

__global__ void k_row_marks(const int32_t *xadj, int32_t n, int32_t *mark) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (xadj[v + 1] > xadj[v]) mark[xadj[v]] = (int32_t)v;
}

struct MaxScanIn {
    const int32_t *mark;
    __device__ int32_t operator()(int64_t i) const { return mark[i]; }
};

// inclusive max-scan is done with a dedicated tile kernel pair (max is not "+")
constexpr int kMB = 256, kMI = 8, kMT = kMB * kMI;

__global__ __launch_bounds__(kMB) void k_tile_max(const int32_t *in, int64_t n, int32_t *partial) {
    __shared__ int32_t tmp[kMB / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kMT;
    int32_t m = -1;
    for (int i = 0; i < kMI; i++) {
        int64_t idx = base + (int64_t)i * kMB + threadIdx.x;
        if (idx < n && in[idx] > m) m = in[idx];
    }
    m = block_max<kMB>(m, tmp);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(kMB) void k_tile_maxscan(int32_t *io, int64_t n, const int32_t *carry) {
    __shared__ int32_t tmp[kMB / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kMT;
    const int64_t mine = base + (int64_t)threadIdx.x * kMI;
    int32_t v[kMI];
    int32_t m = -1;
    for (int i = 0; i < kMI; i++) {
        int64_t idx = mine + i;
        v[i] = idx < n ? io[idx] : -1;
        m = v[i] > m ? v[i] : m;
        v[i] = m;
    }
    // exclusive max over threads: wave inclusive max scan
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int32_t inc = m;
    for (int d = 1; d < kWave; d <<= 1) {
        int32_t y = __shfl_up(inc, d, kWave);
        if (lane >= d && y > inc) inc = y;
    }
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    int32_t pre = carry ? carry[blockIdx.x] : -1;
    for (int i = 0; i < w; i++) pre = tmp[i] > pre ? tmp[i] : pre;
    int32_t ex = __shfl_up(inc, 1, kWave);
    if (lane > 0 && ex > pre) pre = ex;
    for (int i = 0; i < kMI; i++) {
        int64_t idx = mine + i;
        if (idx < n) io[idx] = v[i] > pre ? v[i] : pre;
    }
}

__global__ void k_shift_excl(const int32_t *incl, int64_t n, int32_t *excl) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        excl[i] = i > 0 ? incl[i - 1] : -1;
}

__global__ void k_mark_used(const int32_t *labels, const int32_t *xadj, int32_t n, bool skip_isolated,
                            int32_t *used) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (skip_isolated && xadj[v + 1] == xadj[v]) continue;
        used[labels[v]] = 1;
    }
}

__global__ void k_f2c(const int32_t *labels, const int32_t *xadj, int32_t n, bool skip_isolated,
                      const int32_t *id, const int32_t *vwgt, int32_t *f2c, int64_t *cw) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (skip_isolated && xadj[v + 1] == xadj[v]) {
            f2c[v] = -1;
            continue;
        }
        const int32_t i = id[labels[v]];
        f2c[v] = i;
        atomicAdd((unsigned long long *)&cw[i], (unsigned long long)(vwgt ? vwgt[v] : 1));
    }
}

__global__ void k_cw_out(const int64_t *cw, const int32_t *nc, int32_t *vwgt_c, int32_t *overflow) {
    const int32_t n = *nc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (cw[i] > INT_MAX) *overflow = 1;
        vwgt_c[i] = (int32_t)cw[i];
    }
}

__global__ void k_project(int32_t n, const int32_t *f2c, const int32_t *pc, int32_t *pf) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = f2c[v];
        pf[v] = i >= 0 ? pc[i] : -1;
    }
}

struct CutIn {
    const int32_t *rowof, *adjncy, *adjwgt, *part;
    __device__ int64_t operator()(int64_t e) const {
        return part[rowof[e]] != part[adjncy[e]] ? (adjwgt ? (int64_t)adjwgt[e] : 1) : 0;
    }
};
struct NoOut {
    __device__ void operator()(int64_t, int64_t, int64_t) const {}
};

__global__ void k_halve(int64_t *x) { *x /= 2; }

// ---------------------------------------------------------------- row-grouped contraction

constexpr int kRowWaveMax = 128;    // D_i <= 128: one wave per row
constexpr int kRowBlockMax = 2048;  // D_i <= 2048: one workgroup per row
constexpr int kRowChunk = 2048;     // larger rows: flattened entries per aggregating workgroup
static_assert(kRowWaveMax % kWave == 0, "wave rows: whole entries per lane");

struct RowCtx {
    const int32_t *xadj, *adjncy, *adjwgt, *f2c;
    const int32_t *mstart;   // [nc+1]
    const int32_t *mrow;     // [n_incl] first entry (xadj) of each member, grouped by coarse vertex
    const int32_t *flat;     // [n_incl+1] exclusive prefix of member degrees
    int32_t *tj;             // [nnz] sorted columns of row i at flat[mstart[i]]
    long long *tw;           // [nnz] their weights
    int32_t *rcnt;           // [nc] distinct columns of row i
};

__device__ __forceinline__ uint32_t col_hash(int32_t j) { return (uint32_t)j * 0x9E3779B1u; }

template <typename KeyP, typename ValP>
__device__ __forceinline__ void col_insert(KeyP key, ValP val, uint32_t mask, int lg, int32_t j, long long w) {
    uint32_t h = col_hash(j) >> (32 - lg);
    for (;;) {
        const int32_t prev = atomicCAS(&key[h], -1, j);
        if (prev == -1 || prev == j) break;
        h = (h + 1) & mask;
    }
    atomicAdd((unsigned long long *)&val[h], (unsigned long long)w);
}

// largest p in [lo, hi] with F[p] <= t
__device__ __forceinline__ int32_t upper_pos(const int32_t *F, int32_t lo, int32_t hi, int32_t t) {
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (F[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Entries t = first, first + STRIDE, ... (< tend, at most UB of them) of a
// row. F is the member degree prefix in LDS, relative to the row's first
// entry, for the members whose rows start at mrow[mbase + p], p in [0, pmax].
// Each entry's chain of dependent loads (its member's row start, neighbour,
// neighbour's coarse id) is issued as one batch over the UB entries, so a
// thread waits on memory three times, not three times per entry; the columns
// other than the row itself then go into the row's LDS hash table.
template <int UB, int STRIDE>
__device__ __forceinline__ void gather_insert(const RowCtx &c, const int32_t *F, int32_t mbase, int32_t pmax,
                                              int32_t first, int32_t tend, int32_t i, int32_t *skey,
                                              long long *sval, uint32_t mask, int lg) {
    int32_t x[UB], off[UB], wt[UB];
    int32_t p = 0;
#pragma unroll
    for (int q = 0; q < UB; q++) {
        const int32_t t = first + q * STRIDE;
        if (t < tend) {
            p = upper_pos(F, p, pmax, t);  // t grows: search from the last member
            x[q] = c.mrow[mbase + p];
            off[q] = t - F[p];
        }
    }
#pragma unroll
    for (int q = 0; q < UB; q++)
        if (first + q * STRIDE < tend) x[q] += off[q];  // entry index
#pragma unroll
    for (int q = 0; q < UB; q++)
        if (first + q * STRIDE < tend) {
            wt[q] = c.adjwgt ? c.adjwgt[x[q]] : 1;
            x[q] = c.adjncy[x[q]];
        }
#pragma unroll
    for (int q = 0; q < UB; q++)
        if (first + q * STRIDE < tend) x[q] = c.f2c[x[q]];
#pragma unroll
    for (int q = 0; q < UB; q++)
        if (first + q * STRIDE < tend && x[q] != i) col_insert(skey, sval, mask, lg, x[q], wt[q]);
}

__global__ __launch_bounds__(256) void k_crow_wave(RowCtx c, const int32_t *rows, int32_t count) {
    constexpr int NW = 4, CAP = 2 * kRowWaveMax;
    __shared__ int32_t skey[NW][CAP];
    __shared__ long long sval[NW][CAP];
    __shared__ int32_t sF[NW][kRowWaveMax + 1];
    __shared__ int32_t lj[NW][kRowWaveMax];
    __shared__ long long lw[NW][kRowWaveMax];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int q = lane; q < CAP; q += kWave) {
        skey[w][q] = -1;
        sval[w][q] = 0;
    }
    wave_sync();
    for (int64_t idx = (int64_t)blockIdx.x * NW + w; idx < count; idx += (int64_t)gridDim.x * NW) {
        const int32_t i = rows[idx];
        const int32_t m0 = c.mstart[i], m1 = c.mstart[i + 1];
        const int32_t base = c.flat[m0], D = c.flat[m1] - base, M = m1 - m0;
        for (int q = lane; q <= M; q += kWave) sF[w][q] = c.flat[m0 + q] - base;
        wave_sync();
        int lg = 1;
        while ((1 << lg) < 2 * D) lg++;
        const uint32_t cap = 1u << lg;
        gather_insert<kRowWaveMax / kWave, kWave>(c, sF[w], m0, M - 1, lane, D, i, skey[w], sval[w], cap - 1, lg);
        wave_sync();
        int32_t r = 0;
        for (uint32_t s0 = 0; s0 < cap; s0 += kWave) {
            const uint32_t sl = s0 + lane;
            const bool occ = sl < cap && skey[w][sl] >= 0;
            const uint64_t m = __ballot(occ);
            if (occ) {
                const int32_t pos = r + __popcll(m & lt);
                lj[w][pos] = skey[w][sl];
                lw[w][pos] = sval[w][sl];
            }
            r += __popcll(m);
        }
        wave_sync();
        for (int32_t q = lane; q < r; q += kWave) {
            const int32_t jj = lj[w][q];
            int32_t rank = 0;
            for (int32_t x = 0; x < r; x++) rank += lj[w][x] < jj;
            c.tj[base + rank] = jj;
            c.tw[base + rank] = lw[w][q];
        }
        if (lane == 0) c.rcnt[i] = r;
        for (uint32_t q = lane; q < cap; q += kWave) {
            skey[w][q] = -1;
            sval[w][q] = 0;
        }
        wave_sync();
    }
}

// One workgroup per row. 80 KB of LDS fits two workgroups per CU, so the
// workgroup is wide (kCB threads) to keep enough waves in flight for the
// gathers.
constexpr int kCB = 512;
constexpr int kRankMax = 1024;  // rows with at most this many distinct columns are sorted by counting ranks
static_assert(kRankMax % kCB == 0, "rank sort: whole columns per thread");
static_assert(kRowBlockMax % kCB == 0 && kRowChunk % kCB == 0, "block rows: whole entries per thread");
__global__ __launch_bounds__(kCB) void k_crow_block(RowCtx c, const int32_t *rows, int32_t count) {
    constexpr int CAP = 2 * kRowBlockMax;
    __shared__ int32_t skey[CAP];
    __shared__ long long sval[CAP];
    // sF (member prefix) is only read while gathering and lj (the distinct
    // columns) only written after that, so they share one array; li holds
    // each column's table slot, whose weight is read at the output. This
    // keeps the workgroup under 80 KB: two per CU.
    __shared__ __align__(16) int32_t sFlj[kRowBlockMax + 4];
    __shared__ uint16_t li[kRowBlockMax];
    __shared__ int32_t s_r;
    int32_t *const sF = sFlj, *const lj = sFlj;
    static_assert(2 * kRowBlockMax <= 65536, "slot index fits 16 bits");
    const int lane = lane_id();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int q = threadIdx.x; q < CAP; q += kCB) {
        skey[q] = -1;
        sval[q] = 0;
    }
    __syncthreads();
    for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int32_t i = rows[idx];
        const int32_t m0 = c.mstart[i], m1 = c.mstart[i + 1];
        const int32_t base = c.flat[m0], D = c.flat[m1] - base, M = m1 - m0;
        for (int q = threadIdx.x; q <= M; q += kCB) sF[q] = c.flat[m0 + q] - base;
        if (threadIdx.x == 0) s_r = 0;
        __syncthreads();
        int lg = 1;
        while ((1 << lg) < 2 * D) lg++;
        const uint32_t cap = 1u << lg;
        gather_insert<kRowBlockMax / kCB, kCB>(c, sF, m0, M - 1, threadIdx.x, D, i, skey, sval, cap - 1, lg);
        __syncthreads();
        // compaction of the occupied slots, in any order (the columns are
        // sorted next): one LDS reservation per wave
        for (uint32_t s0 = 0; s0 < cap; s0 += kCB) {
            const uint32_t sl = s0 + threadIdx.x;
            const bool occ = sl < cap && skey[sl] >= 0;
            const uint64_t m = __ballot(occ);
            int32_t wb = 0;
            if (lane == 0 && m) wb = atomicAdd(&s_r, (int32_t)__popcll(m));
            wb = __shfl(wb, 0);
            if (occ) {
                const int32_t pos = wb + (int32_t)__popcll(m & lt);
                lj[pos] = skey[sl];
                li[pos] = (uint16_t)sl;
            }
        }
        __syncthreads();
        const int32_t r = s_r;
        if (r <= kRankMax) {
            // the columns are distinct: each one's rank is the number of
            // smaller ones, counted over broadcast LDS reads (no barriers)
            int32_t jv[kRankMax / kCB], rk[kRankMax / kCB];
#pragma unroll
            for (int q = 0; q < kRankMax / kCB; q++) {
                jv[q] = threadIdx.x + q * kCB < r ? lj[threadIdx.x + q * kCB] : INT_MAX;
                rk[q] = 0;
            }
            const int4 *l4 = reinterpret_cast<const int4 *>(lj);
            int32_t x = 0;
            for (; x + 4 <= r; x += 4) {
                const int4 y = l4[x >> 2];
#pragma unroll
                for (int q = 0; q < kRankMax / kCB; q++)
                    rk[q] += (int32_t)(y.x < jv[q]) + (int32_t)(y.y < jv[q]) + (int32_t)(y.z < jv[q]) +
                             (int32_t)(y.w < jv[q]);
            }
            for (; x < r; x++) {
                const int32_t y = lj[x];
#pragma unroll
                for (int q = 0; q < kRankMax / kCB; q++) rk[q] += (int32_t)(y < jv[q]);
            }
#pragma unroll
            for (int q = 0; q < kRankMax / kCB; q++) {
                const int32_t t = threadIdx.x + q * kCB;
                if (t < r) {
                    c.tj[base + rk[q]] = jv[q];
                    c.tw[base + rk[q]] = sval[li[t]];
                }
            }
        } else {
            int32_t P = 1;
            while (P < r) P <<= 1;
            for (int32_t q = r + threadIdx.x; q < P; q += kCB) lj[q] = INT_MAX;
            __syncthreads();
            // bitonic sort of lj/lw[0, P) by column
            for (int32_t kk = 2; kk <= P; kk <<= 1) {
                for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int32_t q = threadIdx.x; q < P; q += kCB) {
                        const int32_t o = q ^ jj;
                        if (o > q) {
                            const bool up = (q & kk) == 0;
                            const int32_t a = lj[q], b = lj[o];
                            if ((a > b) == up) {
                                lj[q] = b;
                                lj[o] = a;
                                const uint16_t x = li[q];
                                li[q] = li[o];
                                li[o] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int32_t q = threadIdx.x; q < r; q += kCB) {
                c.tj[base + q] = lj[q];
                c.tw[base + q] = sval[li[q]];
            }
        }
        if (threadIdx.x == 0) c.rcnt[i] = r;
        __syncthreads();  // every weight is read before the table is emptied
        for (uint32_t q = threadIdx.x; q < cap; q += kCB) {
            skey[q] = -1;
            sval[q] = 0;
        }
        __syncthreads();
    }
}

// Rows above the LDS classes: chunks of kRowChunk flattened entries, one
// workgroup each, sum their entries per column in an LDS hash and append the
// distinct (row, column) pairs through one reservation per chunk; a radix
// sort then brings equal pairs together and a run reduction merges the chunks
// of a row. The rows are taken in batches of 2^rbits by rank, rbits + jbits
// <= 32, so that a pair's key (rank within the batch << jbits | column) fits
// 32 bits; each batch owns the region of the triple buffers that its chunks'
// capacity spans, and is sorted and reduced on its own.
struct BigRows {
    const int32_t *rows;         // [nb] coarse row ids
    const int32_t *chunk_owner;  // [nchunks] row rank of each chunk
    const int32_t *chunk_first;  // [nb] first chunk of each row
    uint32_t *key;               // [cap] (row rank within its batch << jbits) | column
    int32_t *val;                // [cap] a chunk's partial sum (a coarse weight must fit int32 anyway)
    int32_t *cursor;             // [nbatch] append position within each batch's region
    const int64_t *boff;         // [nbatch] first slot of each batch's region
    int jbits, rbits;
    int32_t *ovf;                // set when a partial sum exceeds int32
};

__global__ __launch_bounds__(kCB) void k_cbig_chunk(RowCtx c, BigRows b) {
    constexpr int CAP = 2 * kRowChunk;
    __shared__ int32_t skey[CAP];
    __shared__ long long sval[CAP];
    __shared__ int32_t sF[kRowChunk + 1];
    __shared__ int32_t rng[2];
    __shared__ int32_t t32[kCB / kWave + 1];
    __shared__ int32_t resv, spos;
    for (int q = threadIdx.x; q < CAP; q += kCB) {
        skey[q] = -1;
        sval[q] = 0;
    }
    const int32_t g = b.chunk_owner[blockIdx.x];
    const int32_t i = b.rows[g];
    const int32_t m0 = c.mstart[i], m1 = c.mstart[i + 1];
    const int32_t base = c.flat[m0], D = c.flat[m1] - base;
    const int32_t t0 = (blockIdx.x - b.chunk_first[g]) * kRowChunk;
    const int32_t t1 = min(D, t0 + kRowChunk);
    if (threadIdx.x == 0) {
        rng[0] = upper_pos(c.flat, m0, m1 - 1, base + t0);
        rng[1] = upper_pos(c.flat, m0, m1 - 1, base + t1 - 1);
    }
    __syncthreads();
    const int32_t plo = rng[0], phi = rng[1];
    if (phi - plo < kRowChunk + 1) {
        // the chunk's members (at most one per entry, unless members without
        // neighbours sit among them) have their prefix staged in LDS
        for (int q = threadIdx.x; q <= phi - plo; q += kCB) sF[q] = c.flat[plo + q] - base;
        __syncthreads();
        gather_insert<kRowChunk / kCB, kCB>(c, sF, plo, phi - plo, t0 + threadIdx.x, t1, i, skey, sval, CAP - 1,
                                            __builtin_ctz(CAP));
    } else {
        int32_t p = plo;
        for (int32_t t = t0 + threadIdx.x; t < t1; t += kCB) {
            p = upper_pos(c.flat, p, phi, base + t);  // t grows per thread: search from the last member
            const int32_t e = c.mrow[p] + (base + t - c.flat[p]);
            const int32_t j = c.f2c[c.adjncy[e]];
            if (j != i) col_insert(skey, sval, CAP - 1, __builtin_ctz(CAP), j, c.adjwgt ? c.adjwgt[e] : 1);
        }
    }
    __syncthreads();
    int32_t cnt = 0;
    for (int q = threadIdx.x; q < CAP; q += kCB) cnt += skey[q] >= 0;
    cnt = block_sum<kCB>(cnt, t32);
    const int32_t bt = g >> b.rbits;
    if (threadIdx.x == 0) {
        resv = cnt ? atomicAdd(&b.cursor[bt], cnt) : 0;
        spos = 0;
    }
    __syncthreads();
    // the pairs go out in any order (a radix sort follows): one LDS
    // reservation per wave within the chunk's range
    const int lane = lane_id();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int q0 = 0; q0 < CAP; q0 += kCB) {
        const int q = q0 + threadIdx.x;
        const bool occ = skey[q] >= 0;
        const uint64_t m = __ballot(occ);
        int32_t wb = 0;
        if (lane == 0 && m) wb = atomicAdd(&spos, (int32_t)__popcll(m));
        wb = __shfl(wb, 0);
        if (occ) {
            const int64_t pos = b.boff[bt] + resv + wb + (int32_t)__popcll(m & lt);
            b.key[pos] = ((uint32_t)(g & ((1 << b.rbits) - 1)) << b.jbits) | (uint32_t)skey[q];
            const long long w = sval[q];
            if (w > INT_MAX) atomicOr(b.ovf, 1);  // the row's total would overflow too
            b.val[pos] = (int32_t)(w > INT_MAX ? INT_MAX : w);
        }
    }
}

struct PairHead {
    const uint32_t *key;
    __device__ bool operator()(int64_t p) const { return p == 0 || key[p] != key[p - 1]; }
};
struct PairHeadEmit {
    int32_t *head;
    __device__ void operator()(int64_t p, int32_t r) const { head[r] = (int32_t)p; }
};
struct ValIn64 {
    const int32_t *v;
    __device__ long long operator()(int64_t p) const { return (long long)v[p]; }
};
struct InclOut64 {
    long long *S;
    __device__ void operator()(int64_t p, long long ex, long long v) const { S[p] = ex + v; }
};

// One batch of big rows, its sorted pairs (key, S: inclusive weight prefix)
// and run heads (positions within the batch's region). Runs are sorted by
// row rank: roff[g] = first run of the batch's rank >= g, for g in [0, nrows].
__global__ void k_cbig_rowoff(const uint32_t *key, const int32_t *head, const int32_t *nruns, int jbits,
                              int32_t nrows, int32_t *roff) {
    const int32_t R = *nruns;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= R; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cur = r < R ? (int64_t)(key[head[r]] >> jbits) : (int64_t)nrows;
        const int64_t prev = r > 0 ? (int64_t)(key[head[r - 1]] >> jbits) : -1;
        for (int64_t g = prev + 1; g <= cur; g++) roff[g] = (int32_t)r;
    }
}

__global__ void k_cbig_place(RowCtx c, const int32_t *rows, const uint32_t *key, int jbits, const int32_t *head,
                             const int32_t *nruns, const int32_t *m_dev, const long long *S, const int32_t *roff,
                             int32_t nrows) {
    const int32_t R = *nruns, m = *m_dev;
    const uint32_t jm = jbits >= 32 ? ~0u : ((1u << jbits) - 1u);
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p0 = head[r], p1 = (r + 1 < R) ? head[r + 1] - 1 : m - 1;
        const uint32_t k = key[p0];
        const int32_t g = (int32_t)(k >> jbits);
        const int32_t i = rows[g];
        const int32_t base = c.flat[c.mstart[i]];
        const int64_t pos = r - roff[g];
        c.tj[base + pos] = (int32_t)(k & jm);
        c.tw[base + pos] = S[p1] - (p0 > 0 ? S[p0 - 1] : 0);
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nrows; g += (int64_t)gridDim.x * blockDim.x)
        c.rcnt[rows[g]] = roff[g + 1] - roff[g];
}

__global__ void k_big_nchunk(RowCtx c, const int32_t *rows, int32_t nb, int32_t *nch) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nb; g += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = rows[g];
        const int32_t D = c.flat[c.mstart[i + 1]] - c.flat[c.mstart[i]];
        nch[g] = (D + kRowChunk - 1) / kRowChunk;
    }
}

__global__ void k_row_counts(const int32_t *f2c, const int32_t *xadj, int32_t n, int32_t *cnt) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = f2c[v];
        if (i >= 0) atomicAdd(&cnt[i], 1);
    }
}

__global__ void k_members(const int32_t *f2c, const int32_t *xadj, int32_t n, const int32_t *mstart, int32_t *fill,
                          int32_t *mrow, int32_t *mdeg) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = f2c[v];
        if (i < 0) continue;
        const int32_t p = mstart[i] + atomicAdd(&fill[i], 1);
        mrow[p] = xadj[v];
        mdeg[p] = xadj[v + 1] - xadj[v];
    }
}

__global__ void k_row_class(const int32_t *mstart, const int32_t *flat, int32_t nc, uint32_t *key, int32_t *val,
                            int32_t *ccount) {
    __shared__ int32_t h[3];
    if (threadIdx.x < 3) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
        // size = max(entries, members): members without neighbours (possible for
        // arbitrary caller labels) still occupy the LDS member-prefix array
        const int32_t D = flat[mstart[i + 1]] - flat[mstart[i]];
        const int32_t M = mstart[i + 1] - mstart[i];
        const int32_t sz = D > M ? D : M;
        const uint32_t k = sz <= kRowWaveMax ? 0u : (sz <= kRowBlockMax ? 1u : 2u);
        key[i] = k;
        val[i] = (int32_t)i;
        atomicAdd(&h[k], 1);
    }
    __syncthreads();
    if (threadIdx.x < 3 && h[threadIdx.x]) atomicAdd(&ccount[threadIdx.x], h[threadIdx.x]);
}

// one wave per big row: its lanes write the row's (possibly thousands of) chunk owners
__global__ __launch_bounds__(256) void k_expand_owner(const int32_t *first, const int32_t *num, int32_t nb,
                                                      int32_t *owner) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; g < nb; g += waves) {
        const int32_t f = first[g], m = num[g];
        for (int32_t q = lane; q < m; q += kWave) owner[f + q] = (int32_t)g;
    }
}

// one wave per coarse row: copy its sorted columns to the output CSR
__global__ void k_copy_rows(RowCtx c, const int32_t *xadj_c, int32_t nc, int32_t *adjncy_c, int32_t *adjwgt_c,
                            int32_t *overflow) {
    const int lane = lane_id();
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    int bad = 0;
    for (int64_t i = wid; i < nc; i += nwaves) {
        const int32_t src = c.flat[c.mstart[i]];
        const int32_t dst = xadj_c[i], r = xadj_c[i + 1] - dst;
        for (int32_t q = lane; q < r; q += kWave) {
            const long long wv = c.tw[src + q];
            bad |= wv > INT_MAX;
            adjncy_c[dst + q] = c.tj[src + q];
            adjwgt_c[dst + q] = (int32_t)wv;
        }
    }
    if (bad) *overflow = 1;
}

struct CountIn {
    const int32_t *r;
    __device__ int32_t operator()(int64_t i) const { return r[i]; }
};
struct CountOut {
    int32_t *x;
    __device__ void operator()(int64_t i, int32_t ex, int32_t) const { x[i] = ex; }
};

}  // namespace

// In-place inclusive max-scan (recursive over tile maxima).
static int maxscan_inclusive(int32_t *io, int64_t n, Scratch &sc) {
    hipStream_t s = sc.stream();
    const int64_t nt = (n + kMT - 1) / kMT;
    if (nt <= 1) {
        hipLaunchKernelGGL(k_tile_maxscan, dim3(1), dim3(kMB), 0, s, io, n, (const int32_t *)nullptr);
        GP_LAUNCH_CHECK();
        return GP_OK;
    }
    int32_t *partial = nullptr, *carry = nullptr;
    GP_TRY(sc.alloc(&partial, nt));
    GP_TRY(sc.alloc(&carry, nt));
    hipLaunchKernelGGL(k_tile_max, dim3(nt), dim3(kMB), 0, s, io, n, partial);
    GP_LAUNCH_CHECK();
    GP_TRY(maxscan_inclusive(partial, nt, sc));
    hipLaunchKernelGGL(k_shift_excl, dim3(grid_for(nt, 256, 65536)), dim3(256), 0, s, partial, nt, carry);
    GP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tile_maxscan, dim3(nt), dim3(kMB), 0, s, io, n, carry);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

int build_rowof(const DevGraph &g, int32_t *rowof, Scratch &sc) {
    hipStream_t s = sc.stream();
    const int64_t nnz = g.nnz;
    if (nnz == 0) return GP_OK;
    GP_HIP(hipMemsetAsync(rowof, 0xFF, sizeof(int32_t) * (size_t)nnz, s));
    hipLaunchKernelGGL(k_row_marks, dim3(grid_for(g.n, 256, 65536)), dim3(256), 0, s, g.xadj, g.n, rowof);
    GP_LAUNCH_CHECK();
    return maxscan_inclusive(rowof, nnz, sc);
}

// Upper bound of the scratch contract() holds at once: the allocations below
// with every coarse count at n, big-row chunk capacity at 2 nnz (chunks of
// kRowChunk entries over rows longer than kRowChunk), runs at that capacity,
// each rounded up to 256 bytes; sort and scan temporaries as for the LP (reusable
// slots grown by 1.25x, at most 6.25 times their final size).
size_t contract_scratch_bound(int64_t n, int64_t nnz) {
    auto R = [](double x) { return (double)((((size_t)(x > 1 ? x : 1)) + 255) & ~(size_t)255); };
    const double N = (double)n, M = (double)nnz, bcap = 2.0 * M + kRowChunk;
    double b = 2 * R(4 * N) + 2 * R(4) + R(8 * N);                          // used, id, counters, c'
    b += R(4 * N) + R(4 * N + 4) + R(4 * N) + 3 * R(4 * N + 4) + R(4);      // counts, starts, members
    b += 2 * R(4 * M) + R(4 * N) + 4 * R(4 * N) + R(12);                     // row buffers, row classes
    b += 2 * R(4 * N) + R(4) + 3 * R(4 * N) + R(4 * N + 4) + R(8 * N);      // big rows: chunk plan, batches
    b += 2 * R(8 * bcap) + 2 * R(4 * bcap) + R(4 * (M / kRowChunk + N));     // big rows: triples
    b += R(8 * bcap) + R(4 * bcap) + R(4);                                   // runs (sized by capacity)
    const double m = std::max(bcap, std::max(N, 1.0));
    const double temps = 6.25 * (m / 4.0) + 6.25 * 2 * 8 * 4 * std::ceil(m / kScanTile) + 128.0 * 1024;
    return (size_t)(b + temps);
}

int contract(const DevGraph &g, const int32_t *labels, bool skip_isolated, CoarseOut &out, Scratch &sc) {
    ScratchScope scope(sc);  // the outputs are caller buffers: all scratch below is internal
    hipStream_t s = sc.stream();
    const int32_t n = g.n;
    out.n = 0;
    out.nnz = 0;
    if (n == 0) {
        GP_HIP(hipMemsetAsync(out.xadj, 0, sizeof(int32_t), s));
        return GP_OK;
    }
    int32_t *used = nullptr, *id = nullptr, *d_nc = nullptr, *flags = nullptr;
    int64_t *cw = nullptr;
    GP_TRY(sc.alloc(&used, n));
    GP_TRY(sc.alloc(&id, n));
    GP_TRY(sc.alloc(&d_nc, 1));
    GP_TRY(sc.alloc(&flags, 1));
    GP_TRY(sc.alloc(&cw, n));
    GP_HIP(hipMemsetAsync(used, 0, sizeof(int32_t) * (size_t)n, s));
    GP_HIP(hipMemsetAsync(cw, 0, sizeof(int64_t) * (size_t)n, s));
    GP_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
    const unsigned gv = grid_for(n, 256, 65536);
    hipLaunchKernelGGL(k_mark_used, dim3(gv), dim3(256), 0, s, labels, g.xadj, n, skip_isolated, used);
    GP_LAUNCH_CHECK();
    GP_TRY((scan<int32_t>(LoadIn<int32_t>{used}, StoreExcl<int32_t>{id}, n, nullptr, d_nc, sc)));
    hipLaunchKernelGGL(k_f2c, dim3(gv), dim3(256), 0, s, labels, g.xadj, n, skip_isolated, id, g.vwgt, out.f2c,
                       cw);
    GP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cw_out, dim3(gv), dim3(256), 0, s, cw, d_nc, out.vwgt, flags);
    GP_LAUNCH_CHECK();
    int32_t nc = 0;
    GP_HIP(hipMemcpyAsync(&nc, d_nc, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));

    const int64_t nnz = g.nnz;
    int32_t nnz_c = 0;
    if (nnz > 0 && nc > 0) {
        // ---- members of each coarse vertex and the prefix of their degrees
        int32_t *cnt = nullptr, *mstart = nullptr, *fill = nullptr, *mrow = nullptr, *mdeg = nullptr,
                *flat = nullptr, *d_ni = nullptr;
        GP_TRY(sc.alloc(&cnt, nc));
        GP_TRY(sc.alloc(&mstart, (size_t)nc + 1));
        GP_TRY(sc.alloc(&fill, nc));
        GP_TRY(sc.alloc(&mrow, n));
        GP_TRY(sc.alloc(&mdeg, n));
        GP_TRY(sc.alloc(&flat, (size_t)n + 1));
        GP_TRY(sc.alloc(&d_ni, 1));
        GP_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)nc, s));
        GP_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * (size_t)nc, s));
        hipLaunchKernelGGL(k_row_counts, dim3(gv), dim3(256), 0, s, out.f2c, g.xadj, n, cnt);
        GP_LAUNCH_CHECK();
        GP_TRY((scan<int32_t>(LoadIn<int32_t>{cnt}, StoreExcl<int32_t>{mstart}, nc, nullptr, mstart + nc, sc)));
        hipLaunchKernelGGL(k_members, dim3(gv), dim3(256), 0, s, out.f2c, g.xadj, n, mstart, fill, mrow, mdeg);
        GP_LAUNCH_CHECK();
        int32_t ni = 0;
        GP_HIP(hipMemcpyAsync(&ni, mstart + nc, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        GP_TRY((scan<int32_t>(LoadIn<int32_t>{mdeg}, StoreExcl<int32_t>{flat}, ni, nullptr, flat + ni, sc)));

        int32_t *tj = nullptr, *rcnt = nullptr;
        long long *tw = nullptr;
        GP_TRY(sc.alloc(&tj, nnz));
        GP_TRY(sc.alloc(&tw, nnz));
        GP_TRY(sc.alloc(&rcnt, nc));
        RowCtx c{g.xadj, g.adjncy, g.adjwgt, out.f2c, mstart, mrow, flat, tj, tw, rcnt};

        // ---- rows by size class (stable, ascending ids inside a class)
        uint32_t *ck = nullptr, *ck2 = nullptr;
        int32_t *cv = nullptr, *cv2 = nullptr, *ccount = nullptr;
        GP_TRY(sc.alloc(&ck, nc));
        GP_TRY(sc.alloc(&ck2, nc));
        GP_TRY(sc.alloc(&cv, nc));
        GP_TRY(sc.alloc(&cv2, nc));
        GP_TRY(sc.alloc(&ccount, 3));
        GP_HIP(hipMemsetAsync(ccount, 0, sizeof(int32_t) * 3, s));
        hipLaunchKernelGGL(k_row_class, dim3(grid_for(nc, 256, 4096)), dim3(256), 0, s, mstart, flat, nc, ck, cv,
                           ccount);
        GP_LAUNCH_CHECK();
        GP_TRY((radix_sort<uint32_t, int32_t>(&ck, &cv, &ck2, &cv2, nc, nullptr, 2, sc)));
        int32_t hc[3];
        GP_HIP(hipMemcpyAsync(hc, ccount, sizeof(hc), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        const int32_t *rows_w = cv, *rows_b = cv + hc[0], *rows_g = cv + hc[0] + hc[1];
        if (hc[0] > 0) {
            hipLaunchKernelGGL(k_crow_wave, dim3(grid_for(hc[0], 4, 65536)), dim3(256), 0, s, c, rows_w, hc[0]);
            GP_LAUNCH_CHECK();
        }
        if (hc[1] > 0) {
            hipLaunchKernelGGL(k_crow_block, dim3(grid_for(hc[1], 1, 8192)), dim3(kCB), 0, s, c, rows_b, hc[1]);
            GP_LAUNCH_CHECK();
        }
        const int32_t nb = hc[2];
        if (nb > 0) {
            int32_t *nch = nullptr, *cfirst = nullptr, *d_tot = nullptr, *cown = nullptr, *cursor = nullptr,
                    *head = nullptr, *d_runs = nullptr, *roff = nullptr;
            GP_TRY(sc.alloc(&nch, nb));
            GP_TRY(sc.alloc(&cfirst, nb));
            GP_TRY(sc.alloc(&d_tot, 1));
            hipLaunchKernelGGL(k_big_nchunk, dim3(grid_for(nb, 256, 1024)), dim3(256), 0, s, c, rows_g, nb, nch);
            GP_LAUNCH_CHECK();
            GP_TRY((scan<int32_t>(LoadIn<int32_t>{nch}, StoreExcl<int32_t>{cfirst}, nb, nullptr, d_tot, sc)));
            int32_t nchunks = 0;
            GP_HIP(hipMemcpyAsync(&nchunks, d_tot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            std::vector<int32_t> hfirst(nb);
            GP_HIP(hipMemcpyAsync(hfirst.data(), cfirst, sizeof(int32_t) * (size_t)nb, hipMemcpyDeviceToHost, s));
            GP_HIP(hipStreamSynchronize(s));
            const int64_t bcap = (int64_t)nchunks * kRowChunk;
            const int jbits = bits_for(nc - 1) > 0 ? bits_for(nc - 1) : 1;
            const int gbits = bits_for(nb - 1) > 0 ? bits_for(nb - 1) : 1;
            const int rbits = std::max(1, std::min(gbits, 32 - jbits));
            const int32_t rows_per = (int32_t)1 << rbits;
            const int32_t nbatch = (nb + rows_per - 1) / rows_per;
            // batch t: ranks [t * rows_per, +rows_per), slots [boff[t], boff[t + 1])
            std::vector<int64_t> hoff(nbatch + 1);
            for (int32_t t = 0; t < nbatch; t++) hoff[t] = (int64_t)hfirst[(size_t)t * rows_per] * kRowChunk;
            hoff[nbatch] = bcap;
            uint32_t *bk = nullptr, *bk2 = nullptr;
            int32_t *bv = nullptr, *bv2 = nullptr;
            long long *S = nullptr;
            int64_t *boff = nullptr;
            GP_TRY(sc.alloc(&bk, bcap));
            GP_TRY(sc.alloc(&bk2, bcap));
            GP_TRY(sc.alloc(&bv, bcap));
            GP_TRY(sc.alloc(&bv2, bcap));
            GP_TRY(sc.alloc(&S, bcap));
            GP_TRY(sc.alloc(&head, bcap));
            GP_TRY(sc.alloc(&cursor, nbatch));
            GP_TRY(sc.alloc(&d_runs, nbatch));
            GP_TRY(sc.alloc(&roff, (size_t)nb + nbatch));
            GP_TRY(sc.alloc(&boff, nbatch));
            GP_HIP(hipMemcpyAsync(boff, hoff.data(), sizeof(int64_t) * (size_t)nbatch, hipMemcpyHostToDevice, s));
            GP_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (size_t)nbatch, s));
            GP_HIP(hipMemsetAsync(d_runs, 0, sizeof(int32_t) * (size_t)nbatch, s));
            std::vector<int32_t> hm(nbatch, 0);
            if (nchunks > 0) {  // rows whose members have no neighbours have no chunks
                GP_TRY(sc.alloc(&cown, nchunks));
                hipLaunchKernelGGL(k_expand_owner, dim3(grid_for(nb, 4, 4096)), dim3(256), 0, s, cfirst, nch, nb,
                                   cown);
                GP_LAUNCH_CHECK();
                BigRows br{rows_g, cown, cfirst, bk, bv, cursor, boff, jbits, rbits, flags};
                hipLaunchKernelGGL(k_cbig_chunk, dim3(nchunks), dim3(kCB), 0, s, c, br);
                GP_LAUNCH_CHECK();
                GP_HIP(hipMemcpyAsync(hm.data(), cursor, sizeof(int32_t) * (size_t)nbatch, hipMemcpyDeviceToHost, s));
                GP_HIP(hipStreamSynchronize(s));  // the host vectors outlive every copy queued above
            }
            for (int32_t t = 0; t < nbatch; t++) {
                const int64_t o = hoff[t], cap = hoff[t + 1] - o;
                const int32_t nrows = std::min(rows_per, nb - t * rows_per);
                const int kbits = jbits + (bits_for(nrows - 1) > 0 ? bits_for(nrows - 1) : 1);
                uint32_t *k1 = bk + o, *k2 = bk2 + o;
                int32_t *v1 = bv + o, *v2 = bv2 + o;
                if (hm[t] > 0) {
                    // sized by the capacity, with the live count on the device: the
                    // number of triples depends on which members share a chunk, and
                    // members are grouped by atomics in no fixed order, so sizing by
                    // the count would make the call's scratch vary from run to run
                    // (the result does not: the triples are sorted and summed)
                    GP_TRY((radix_sort<uint32_t, int32_t>(&k1, &v1, &k2, &v2, cap, cursor + t, kbits, sc)));
                    GP_TRY((scan<long long>(ValIn64{v1}, InclOut64{S + o}, cap, cursor + t, (long long *)nullptr, sc)));
                    GP_TRY(compact(PairHead{k1}, PairHeadEmit{head + o}, cap, cursor + t, d_runs + t, sc));
                }
                int32_t *ro = roff + (int64_t)t * (rows_per + 1);
                hipLaunchKernelGGL(k_cbig_rowoff, dim3(grid_for((int64_t)hm[t] + 1, 256, 65536)), dim3(256), 0, s,
                                   k1, head + o, d_runs + t, jbits, nrows, ro);
                GP_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_cbig_place, dim3(grid_for((int64_t)hm[t] + nrows, 256, 65536)), dim3(256), 0, s, c,
                                   rows_g + (int64_t)t * rows_per, k1, jbits, head + o, d_runs + t, cursor + t, S + o,
                                   ro, nrows);
                GP_LAUNCH_CHECK();
            }
        }
        // ---- coarse row offsets and the compacted rows
        int32_t *d_nnzc = nullptr;
        GP_TRY(sc.alloc(&d_nnzc, 1));
        GP_TRY((scan<int32_t>(CountIn{rcnt}, CountOut{out.xadj}, nc, nullptr, d_nnzc, sc)));
        GP_HIP(hipMemcpyAsync(out.xadj + nc, d_nnzc, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_copy_rows, dim3(grid_for((int64_t)nc * kWave, 256, 65536)), dim3(256), 0, s, c, out.xadj,
                           nc, out.adjncy, out.adjwgt, flags);
        GP_LAUNCH_CHECK();
        GP_HIP(hipMemcpyAsync(&nnz_c, d_nnzc, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    } else {
        GP_HIP(hipMemsetAsync(out.xadj, 0, sizeof(int32_t) * (size_t)(nc + 1), s));
    }
    int32_t ovf = 0;
    GP_HIP(hipMemcpyAsync(&ovf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    if (ovf) {
        set_error("contract: a coarse vertex or edge weight exceeds int32");
        return GP_ERR_OVERFLOW;
    }
    out.n = nc;
    out.nnz = nnz_c;
    return GP_OK;
}

int project(int32_t n, const int32_t *f2c, const int32_t *part_coarse, int32_t *part_fine, hipStream_t s) {
    if (n <= 0) return GP_OK;
    hipLaunchKernelGGL(k_project, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, f2c, part_coarse, part_fine);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

int cut_dev(const DevGraph &g, const int32_t *part, const int32_t *rowof, int64_t *cut_out, Scratch &sc) {
    hipStream_t s = sc.stream();
    if (g.nnz == 0) {
        GP_HIP(hipMemsetAsync(cut_out, 0, sizeof(int64_t), s));
        return GP_OK;
    }
    int32_t *ro = const_cast<int32_t *>(rowof);
    if (!ro) {
        GP_TRY(sc.alloc(&ro, g.nnz));
        GP_TRY(build_rowof(g, ro, sc));
    }
    GP_TRY((reduce<int64_t>(CutIn{ro, g.adjncy, g.adjwgt, part}, g.nnz, nullptr, cut_out, sc)));
    hipLaunchKernelGGL(k_halve, dim3(1), dim3(1), 0, s, cut_out);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

}  // namespace gp
