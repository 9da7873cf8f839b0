// initpart.hip — initial partitioning of the coarsest graph on the GPU
// (§III-B: recursive bisection into ceil(k/2) / floor(k/2) blocks, best of
// several independent tries, §IV-B), plus placement of vertices without
// neighbours.
//
// Bisection of a vertex set S with k_S blocks grows the left side by a FIFO
// breadth-first search inside S from a hashed start vertex until it weighs at
// least ceil(c(S) * ceil(k_S/2) / k_S). The search runs in one workgroup, one
// BFS level at a time, but reproduces the FIFO queue order exactly: a vertex
// discovered by several frontier vertices belongs to the earliest (frontier
// position, adjacency position) pair, found with an atomicMin over edge ranks.
// All subproblems of one recursion depth, for all tries, run as one launch.
//
// Every try is then refined by LP at once, on the disjoint union of the tries
// (try a owns vertices a*n.. and labels a*k..): LP never mixes components and
// a component that went idle twice stays idle, so each try gets exactly the
// result it would get alone. Then each try is greedily rebalanced by one
// workgroup, and the best try by (imbalanced, cut, index) is kept.
#include <algorithm>
#include <array>
#include <climits>

#include "contract.hpp"
#include "initpart.hpp"
#include "prims.hpp"

namespace gp {

namespace {

constexpr int kBB = 1024;  // bisection workgroup

// splitmix64 finaliser of x + gamma (Steele, Lea & Flood 2014)
__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t vw(const int32_t *vwgt, int32_t v) { return vwgt ? vwgt[v] : 1; }

struct BisectArgs {
    int32_t n;
    const int32_t *xadj, *adjncy, *vwgt;
    int32_t *blk;    // [attempts * n] global block ids (graph block base + local), -1 = not taking part
    int32_t *mark;   // [attempts * n]
    int32_t *claim;  // [attempts * n]
    int32_t *slist;  // per workgroup region (its graph's size)
    int32_t *order;  // per workgroup region
    int32_t *pre;    // per workgroup region (+1) frontier degree prefix
    const int64_t *reg;  // [nsub] region offset of subproblem (per attempt: + attempt * regtot)
    int64_t regtot;
    const int32_t *sub_g, *sub_base, *sub_ks;  // graph, local block base, blocks of each subproblem
    const int32_t *voff, *kbase;               // graph vertex ranges and block bases
    int32_t nsub;
    uint64_t seed;
};

// finds the frontier position of edge rank r: largest i with pre[i] <= r
__device__ __forceinline__ int32_t frontier_pos(const int32_t *pre, int32_t f, int32_t r) {
    int32_t lo = 0, hi = f - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBB) void k_bisect(BisectArgs a) {
    __shared__ int64_t t64[kBB / kWave + 1];
    __shared__ int32_t t32[kBB / kWave + 1];
    __shared__ int32_t sh_tail, sh_stop, sh_found;
    const int attempt = blockIdx.x / a.nsub, sp = blockIdx.x % a.nsub;
    const int32_t gr = a.sub_g[sp];
    const int32_t lbase = a.sub_base[sp], ks = a.sub_ks[sp], kl = (ks + 1) / 2;
    const int32_t base = a.kbase[gr] + lbase;  // global block id of this subproblem
    const int32_t n = a.n;
    const int32_t vlo = a.voff[gr], vhi = a.voff[gr + 1];
    int32_t *blk = a.blk + (int64_t)attempt * n;
    int32_t *mark = a.mark + (int64_t)attempt * n;
    int32_t *claim = a.claim + (int64_t)attempt * n;
    const int64_t rg = (int64_t)attempt * a.regtot + a.reg[sp];
    int32_t *slist = a.slist + rg;
    int32_t *order = a.order + rg;
    int32_t *pre = a.pre + rg + sp + (int64_t)attempt * a.nsub;

    // ---- S in ascending order, its weight; reset marks and claims
    int32_t size = 0;
    int64_t cs = 0;
    for (int32_t v0 = vlo; v0 < vhi; v0 += kBB) {
        const int32_t v = v0 + threadIdx.x;
        const bool in = v < vhi && blk[v] == base;
        int32_t tot;
        const int32_t ex = block_excl_scan<kBB>((int32_t)in, t32, &tot);
        if (in) {
            slist[size + ex] = v;
            mark[v] = 0;
            claim[v] = INT_MAX;
            cs += vw(a.vwgt, v);
        }
        size += tot;
    }
    cs = block_sum<kBB>(cs, t64);
    if (size == 0) return;
    const int64_t q = cs / ks, rm = cs % ks;
    const int64_t target = q * kl + (rm * kl + ks - 1) / ks;
    const uint64_t h = splitmix(splitmix(splitmix(splitmix(a.seed) ^ (uint64_t)attempt) ^ (uint64_t)lbase) ^
                                (uint64_t)ks);
    const int32_t start = slist[h % (uint64_t)size];
    __syncthreads();
    if (threadIdx.x == 0) {
        order[0] = start;
        mark[start] = 1;
    }
    __syncthreads();

    int32_t head = 0, tail = 1, scanp = 0, stop = -1;
    int64_t cum = 0;
    for (;;) {
        // ---- pops of this frontier: first position where the left side reaches the target
        const int32_t f = tail - head;
        for (int32_t c0 = 0; c0 < f && stop < 0; c0 += kBB) {
            const int32_t i = c0 + threadIdx.x;
            const int64_t w = i < f ? vw(a.vwgt, order[head + i]) : 0;
            int64_t tot;
            const int64_t ex = block_excl_scan<kBB>(w, t64, &tot);
            const int32_t hit = (i < f && cum + ex + w >= target) ? i : INT_MAX;
            const int32_t first = block_min<kBB>(hit, t32);
            if (first != INT_MAX) stop = head + first;
            cum += tot;
        }
        if (stop >= 0) break;
        // ---- expand: degree prefix over the frontier (edges inside S only are claimed)
        int32_t ef = 0;
        for (int32_t c0 = 0; c0 < f; c0 += kBB) {
            const int32_t i = c0 + threadIdx.x;
            int32_t d = 0;
            if (i < f) {
                const int32_t v = order[head + i];
                d = a.xadj[v + 1] - a.xadj[v];
            }
            int32_t tot;
            const int32_t ex = block_excl_scan<kBB>(d, t32, &tot);
            if (i < f) pre[i] = ef + ex;
            ef += tot;
        }
        __syncthreads();
        for (int32_t r = threadIdx.x; r < ef; r += kBB) {
            const int32_t i = frontier_pos(pre, f, r);
            const int32_t v = order[head + i];
            const int32_t u = a.adjncy[a.xadj[v] + (r - pre[i])];
            if (blk[u] == base && !mark[u]) atomicMin(&claim[u], r);
        }
        __syncthreads();
        int32_t nt = tail;
        for (int32_t r0 = 0; r0 < ef; r0 += kBB) {
            const int32_t r = r0 + threadIdx.x;
            int32_t u = -1;
            if (r < ef) {
                const int32_t i = frontier_pos(pre, f, r);
                const int32_t v = order[head + i];
                const int32_t cand = a.adjncy[a.xadj[v] + (r - pre[i])];
                if (blk[cand] == base && !mark[cand] &&
                    __hip_atomic_load(&claim[cand], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == r)
                    u = cand;
            }
            int32_t tot;
            const int32_t ex = block_excl_scan<kBB>((int32_t)(u >= 0), t32, &tot);
            if (u >= 0) order[nt + ex] = u;
            nt += tot;
        }
        __syncthreads();
        for (int32_t p = tail + threadIdx.x; p < nt; p += kBB) mark[order[p]] = 1;
        __syncthreads();
        head = tail;
        tail = nt;
        if (head == tail) {
            // queue ran dry: smallest unmarked vertex of S
            int32_t found = INT_MAX;
            while (found == INT_MAX && scanp < size) {
                const int32_t i = scanp + threadIdx.x;
                const int32_t hit = (i < size && !mark[slist[i]]) ? i : INT_MAX;
                found = block_min<kBB>(hit, t32);
                if (found == INT_MAX) scanp += kBB;
            }
            if (found == INT_MAX) {  // cannot happen: target <= c(S)
                stop = tail - 1;
                break;
            }
            scanp = found;
            if (threadIdx.x == 0) {
                order[tail] = slist[found];
                mark[slist[found]] = 1;
            }
            __syncthreads();
            tail++;
        }
    }
    // ---- left side = order[0..stop]; the rest of S gets base + kl
    for (int32_t i = threadIdx.x; i < size; i += kBB) blk[slist[i]] = base + kl;
    __syncthreads();
    for (int32_t p = threadIdx.x; p <= stop; p += kBB) blk[order[p]] = base;
}

// ---- 2-way FM after a bisection (§III-B: the bisection is improved by local
// search). One workgroup per (try, subproblem), over S = the vertices of both
// new sides (base: left, base + kl: right); only edges inside S count. A pass:
// gains from scratch (edge-parallel over S, integer atomics), then moves one
// at a time: the unlocked vertex of largest gain whose receiving side stays
// within (blocks it will hold) * L_max, ties to the lowest id, found by a
// block-wide max over S; its neighbours' gains change by -/+2w. A pass stops
// when nothing may move or after kFmIdle moves without a new best running
// gain; moves past the shortest best prefix are undone. Passes repeat until
// one gains nothing. Side, lock and gain words are read with agent-scope loads
// (they are written by this workgroup's atomics and stores within the pass).
constexpr int kFmIdle = 50;

struct FmArgs {
    const int32_t *xadj, *adjncy, *adjwgt, *vwgt;
    int32_t n;
    int32_t *blk;      // [attempts * n]
    int32_t *lock;     // [attempts * n]
    int64_t *gain;     // [attempts * n]
    int32_t *pos;      // [attempts * n] index in S (valid only for vertices of S)
    int32_t *slist;    // per workgroup region: S ascending
    int32_t *log;      // per workgroup region: moves of the pass
    const int64_t *reg;
    int64_t regtot;
    const int32_t *sub_g, *sub_base, *sub_ks;
    const int32_t *voff, *kbase;
    const int64_t *lmax;  // [G]
    int32_t nsub;
    int32_t passes;
    int32_t wide;  // connection sums may exceed 32 bits: gains stay in global int64 words
};

template <typename T>
__device__ __forceinline__ T ld_dev(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kFmLds = 16384;  // largest S searched in LDS (9 bytes per vertex)

__global__ __launch_bounds__(kBB) void k_fm(FmArgs a) {
    __shared__ int64_t t64[kBB / kWave + 1];
    __shared__ int32_t t32[kBB / kWave + 1];
    __shared__ int32_t sg_[kFmLds];  // gain
    __shared__ int32_t sw_[kFmLds];  // vertex weight
    __shared__ uint8_t sf_[kFmLds];  // bit 0: right side, bit 1: locked
    __shared__ unsigned long long tu[kBB / kWave + 1];
    static_assert(kFmLds <= 0xFFFF + 1, "positions are packed into 16 bits");
    const int attempt = blockIdx.x / a.nsub, sp = blockIdx.x % a.nsub;
    const int32_t gr = a.sub_g[sp];
    const int32_t ks = a.sub_ks[sp], kl = (ks + 1) / 2;
    const int32_t base = a.kbase[gr] + a.sub_base[sp], right = base + kl;
    const int64_t U0 = (int64_t)kl * a.lmax[gr], U1 = (int64_t)(ks - kl) * a.lmax[gr];
    const int32_t n = a.n;
    const int32_t vlo = a.voff[gr], vhi = a.voff[gr + 1];
    int32_t *blk = a.blk + (int64_t)attempt * n;
    int32_t *lock = a.lock + (int64_t)attempt * n;
    int64_t *gain = a.gain + (int64_t)attempt * n;
    const int64_t rg = (int64_t)attempt * a.regtot + a.reg[sp];
    int32_t *slist = a.slist + rg;
    int32_t *log = a.log + rg;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;

    // ---- S ascending
    int32_t size = 0;
    for (int32_t v0 = vlo; v0 < vhi; v0 += kBB) {
        const int32_t v = v0 + threadIdx.x;
        const bool in = v < vhi && (blk[v] == base || blk[v] == right);
        int32_t tot;
        const int32_t ex = block_excl_scan<kBB>((int32_t)in, t32, &tot);
        if (in) slist[size + ex] = v;
        size += tot;
    }
    if (size == 0) return;
    __syncthreads();

    if (size <= kFmLds && !a.wide) {
        // ---- the same search with gains, weights and side/lock flags in LDS,
        // indexed by position in S (ascending ids, so the lowest position is
        // the lowest id); neighbours are found through pos[] once blk[] says
        // they belong to S.
        const int32_t *pos = a.pos + (int64_t)attempt * n;
        for (int32_t i = threadIdx.x; i < size; i += kBB) {
            const int32_t v = slist[i];
            a.pos[(int64_t)attempt * n + v] = i;
            sw_[i] = (int32_t)vw(a.vwgt, v);
            sf_[i] = blk[v] == right ? 1 : 0;
        }
        __syncthreads();
        for (int32_t pass = 0; pass < a.passes; pass++) {
            int64_t w0 = 0, wall = 0;
            for (int32_t i = threadIdx.x; i < size; i += kBB) {
                wall += sw_[i];
                if (!(sf_[i] & 1)) w0 += sw_[i];
                sf_[i] &= 1;
                sg_[i] = 0;
            }
            w0 = block_sum<kBB>(w0, t64);
            wall = block_sum<kBB>(wall, t64);
            int64_t W0 = w0, W1 = wall - w0;
            __syncthreads();
            for (int32_t i = wid; i < size; i += kBB / kWave) {  // one wave per vertex
                const int32_t v = slist[i];
                const uint8_t sv = sf_[i] & 1;
                int32_t acc = 0;
                for (int32_t e = a.xadj[v] + lane; e < a.xadj[v + 1]; e += kWave) {
                    const int32_t u = a.adjncy[e];
                    const int32_t bu = blk[u];
                    if (u == v || (bu != base && bu != right)) continue;
                    const int32_t w = a.adjwgt ? a.adjwgt[e] : 1;
                    acc += (sf_[pos[u]] & 1) != sv ? w : -w;
                }
                acc = wave_sum(acc);
                if (lane == 0) sg_[i] = acc;
            }
            __syncthreads();
            int64_t run = 0, best = 0;
            int32_t len = 0, best_len = 0, idle = 0;
            for (;;) {
                // one key per candidate, largest wins: gain (sign bit flipped
                // for unsigned order), then the lowest position, then its side
                // (so no thread reads the mover's flags after the max); 0 = none
                unsigned long long bk = 0;
                for (int32_t i = threadIdx.x; i < size; i += kBB) {
                    const uint8_t f = sf_[i];
                    const bool left = !(f & 1);
                    if ((f & 2) || (left ? W1 : W0) + sw_[i] > (left ? U1 : U0)) continue;
                    const unsigned long long key =
                        ((unsigned long long)((uint32_t)sg_[i] ^ 0x80000000u) << 32) |
                        ((unsigned long long)(0xFFFFu - (uint32_t)i) << 1) | (unsigned long long)(f & 1);
                    bk = key > bk ? key : bk;
                }
                bk = block_max<kBB>(bk, tu);
                if (bk == 0) break;
                const int64_t gmax = (int32_t)((uint32_t)(bk >> 32) ^ 0x80000000u);
                const int32_t i = (int32_t)(0xFFFFu - (uint32_t)((bk >> 1) & 0xFFFFu));
                const int32_t v = slist[i];
                const uint8_t to = (uint8_t)((bk & 1) ^ 1);
                if (to) {
                    W0 -= sw_[i];
                    W1 += sw_[i];
                } else {
                    W1 -= sw_[i];
                    W0 += sw_[i];
                }
                if (threadIdx.x == 0) {
                    sf_[i] = to | 2;
                    log[len] = i;
                }
                for (int32_t e = a.xadj[v] + threadIdx.x; e < a.xadj[v + 1]; e += kBB) {
                    const int32_t u = a.adjncy[e];
                    const int32_t bu = blk[u];
                    if (u == v || (bu != base && bu != right)) continue;
                    const int32_t j = pos[u];
                    const int32_t w = a.adjwgt ? a.adjwgt[e] : 1;
                    atomicAdd(&sg_[j], (sf_[j] & 1) == to ? -2 * w : 2 * w);
                }
                __syncthreads();
                len++;
                run += gmax;
                if (run > best) {
                    best = run;
                    best_len = len;
                    idle = 0;
                } else if (++idle >= kFmIdle) {
                    break;
                }
            }
            for (int32_t q = best_len + threadIdx.x; q < len; q += kBB) sf_[log[q]] ^= 1;
            __syncthreads();
            if (best <= 0) break;
        }
        for (int32_t i = threadIdx.x; i < size; i += kBB) blk[slist[i]] = (sf_[i] & 1) ? right : base;
        return;
    }

    for (int32_t pass = 0; pass < a.passes; pass++) {
        // ---- side weights, locks and gains from scratch
        int64_t w0 = 0, wall = 0;
        for (int32_t i = threadIdx.x; i < size; i += kBB) {
            const int32_t v = slist[i];
            const int64_t c = vw(a.vwgt, v);
            wall += c;
            if (ld_dev(&blk[v]) == base) w0 += c;
            lock[v] = 0;
        }
        w0 = block_sum<kBB>(w0, t64);
        wall = block_sum<kBB>(wall, t64);
        int64_t W0 = w0, W1 = wall - w0;
        for (int32_t i = wid; i < size; i += kBB / kWave) {  // one wave per vertex
            const int32_t v = slist[i];
            const int32_t bv = ld_dev(&blk[v]);
            int64_t acc = 0;
            for (int32_t e = a.xadj[v] + lane; e < a.xadj[v + 1]; e += kWave) {
                const int32_t u = a.adjncy[e];
                const int32_t bu = ld_dev(&blk[u]);
                if (u == v || (bu != base && bu != right)) continue;
                const int64_t w = a.adjwgt ? a.adjwgt[e] : 1;
                acc += bu != bv ? w : -w;
            }
            acc = wave_sum(acc);
            if (lane == 0) gain[v] = acc;
        }
        __threadfence();  // locks and gains reach L2 before the agent-scope loads below
        __syncthreads();

        int64_t run = 0, best = 0;
        int32_t len = 0, best_len = 0, idle = 0;
        for (;;) {
            // ---- the unlocked vertex of largest gain that fits, lowest id on ties
            int64_t bg = INT64_MIN;
            int32_t bv = INT_MAX;
            for (int32_t i = threadIdx.x; i < size; i += kBB) {
                const int32_t v = slist[i];
                if (ld_dev(&lock[v])) continue;
                const bool left = ld_dev(&blk[v]) == base;
                if ((left ? W1 : W0) + vw(a.vwgt, v) > (left ? U1 : U0)) continue;
                const int64_t gv = ld_dev(&gain[v]);
                if (gv > bg) {  // ascending v per thread: the first of equal gains is the lowest
                    bg = gv;
                    bv = v;
                }
            }
            const int64_t gmax = block_max<kBB>(bg, t64);
            if (gmax == INT64_MIN) break;
            const int32_t v = block_min<kBB>(bg == gmax ? bv : INT_MAX, t32);
            const bool left = ld_dev(&blk[v]) == base;
            const int32_t to = left ? right : base;
            const int64_t c = vw(a.vwgt, v);
            if (left) {
                W0 -= c;
                W1 += c;
            } else {
                W1 -= c;
                W0 += c;
            }
            __syncthreads();  // every thread has read v's side
            if (threadIdx.x == 0) {
                blk[v] = to;
                lock[v] = 1;
                log[len] = v;
            }
            for (int32_t e = a.xadj[v] + threadIdx.x; e < a.xadj[v + 1]; e += kBB) {
                const int32_t u = a.adjncy[e];
                const int32_t bu = ld_dev(&blk[u]);
                if (u == v || (bu != base && bu != right)) continue;
                const int64_t w = a.adjwgt ? a.adjwgt[e] : 1;
                atomicAdd((unsigned long long *)&gain[u], (unsigned long long)(bu == to ? -2 * w : 2 * w));
            }
            __threadfence();
            __syncthreads();
            len++;
            run += gmax;
            if (run > best) {
                best = run;
                best_len = len;
                idle = 0;
            } else if (++idle >= kFmIdle) {
                break;
            }
        }
        // ---- undo the moves past the best prefix (each vertex moved at most once)
        for (int32_t i = best_len + threadIdx.x; i < len; i += kBB) {
            const int32_t v = ld_dev(&log[i]);
            blk[v] = ld_dev(&blk[v]) == base ? right : base;
        }
        __threadfence();
        __syncthreads();
        if (best <= 0) break;
    }
}

__global__ void k_init_blk(int32_t n, int32_t attempts, const int32_t *xadj, bool skip_isolated, const int32_t *gid,
                           const int32_t *kbase, int32_t *blk) {
    const int64_t N = (int64_t)n * attempts;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i % n);
        blk[i] = (skip_isolated && xadj[v + 1] == xadj[v]) ? -1 : kbase[gid[v]];
    }
}

// Disjoint union of the tries: try c owns vertices c*n.. and labels c*Ktot..
__global__ void k_union(int32_t n, int32_t nnz, int32_t attempts, int32_t ktot, const int32_t *xadj,
                        const int32_t *adjncy, const int32_t *adjwgt, const int32_t *vwgt, const int32_t *blk,
                        int32_t *uxadj, int32_t *uadj, int32_t *uw, int32_t *uvw, int32_t *ulab) {
    const int64_t NV = (int64_t)n * attempts, NE = (int64_t)nnz * attempts;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= NV; i += stride) {
        if (i == NV) {
            uxadj[NV] = (int32_t)NE;
            continue;
        }
        const int64_t c = i / n, v = i % n;
        uxadj[i] = (int32_t)(c * nnz + xadj[v]);
        if (uvw) uvw[i] = vwgt[v];
        const int32_t b = blk[i];
        ulab[i] = b >= 0 ? (int32_t)(c * ktot + b) : -1;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < NE; e += stride) {
        const int64_t c = e / nnz, ee = e % nnz;
        uadj[e] = (int32_t)(c * n + adjncy[ee]);
        if (uw) uw[e] = adjwgt[ee];
    }
}

// capacity of union label c*Ktot + kbase[g] + b is lmax[g]
__global__ void k_label_caps(int32_t attempts, int32_t ktot, int32_t G, const int32_t *kbase, const int64_t *lmax,
                             int64_t *cap) {
    const int64_t N = (int64_t)attempts * ktot;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = (int32_t)(i % ktot);
        int32_t lo = 0, hi = G - 1;  // graph with kbase[g] <= b < kbase[g+1]
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (kbase[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        cap[i] = lmax[lo];
    }
}

// One workgroup per (try, graph): while a block exceeds lmax apply the move
// (v, t) of maximum gain conn(v,t) - conn(v,P(v)) with v in an overloaded
// block and B[t] + c(v) <= lmax; ties -> lowest v, then lowest t.
constexpr int kRB = 512;
__global__ __launch_bounds__(kRB) void k_rebalance(int32_t n, int32_t G, int32_t ktot, const int32_t *voff,
                                                   const int32_t *kbase, const int64_t *lmaxv, const int32_t *xadj,
                                                   const int32_t *adjncy, const int32_t *adjwgt,
                                                   const int32_t *vwgt, int32_t *ulab, int32_t *balanced,
                                                   int32_t kmax) {
    extern __shared__ int64_t dyn[];
    constexpr int NW = kRB / kWave;
    const int a = blockIdx.x / G, gr = blockIdx.x % G;
    const int32_t k = kbase[gr + 1] - kbase[gr];
    const int64_t lmax = lmaxv[gr];
    int64_t *B = dyn;                 // [k]
    int64_t *conn = dyn + kmax;       // [NW][kmax]
    __shared__ int64_t bg[NW];
    __shared__ int32_t bv[NW], bt[NW];
    __shared__ int32_t s_over;
    const int32_t *ux = xadj;  // union graph: try a is vertices [a*n, (a+1)*n)
    int32_t *lab = ulab;
    const int32_t v0 = a * n + voff[gr], nv = voff[gr + 1] - voff[gr];
    const int32_t l0 = a * ktot + kbase[gr];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int64_t *cw = conn + (int64_t)w * kmax;
    for (int b = threadIdx.x; b < k; b += kRB) B[b] = 0;
    __syncthreads();
    for (int32_t v = threadIdx.x; v < nv; v += kRB) {
        const int32_t L = lab[v0 + v];
        if (L >= 0) atomicAdd((unsigned long long *)&B[L - l0], (unsigned long long)vw(vwgt, v0 + v));
    }
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) {
            int over = 0;
            for (int b = 0; b < k; b++) over |= B[b] > lmax;
            s_over = over;
        }
        __syncthreads();
        if (!s_over) {
            if (threadIdx.x == 0) balanced[blockIdx.x] = 1;
            return;
        }
        int64_t best_g = LLONG_MIN;
        int32_t best_v = INT_MAX, best_t = INT_MAX;
        for (int32_t v = w; v < nv; v += NW) {
            const int32_t L = lab[v0 + v];
            if (L < 0 || B[L - l0] <= lmax) continue;  // wave-uniform
            const int32_t pv = L - l0;
            for (int b = lane; b < k; b += kWave) cw[b] = 0;
            wave_sync();
            for (int32_t e = ux[v0 + v] + lane; e < ux[v0 + v + 1]; e += kWave) {
                const int32_t u = adjncy[e];
                const int32_t Lu = lab[u];
                atomicAdd((unsigned long long *)&cw[Lu - l0], (unsigned long long)(adjwgt ? adjwgt[e] : 1));
            }
            wave_sync();
            const int64_t cv = vw(vwgt, v0 + v);
            const int64_t own = cw[pv];
            for (int t = lane; t < k; t += kWave) {
                if (t == pv || B[t] + cv > lmax) continue;
                const int64_t g = cw[t] - own;
                if (g > best_g || (g == best_g && (v < best_v || (v == best_v && t < best_t)))) {
                    best_g = g;
                    best_v = v;
                    best_t = t;
                }
            }
            wave_sync();
        }
        // reduce (gain desc, v asc, t asc) over the wave, then the block
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const int64_t og = __shfl_xor(best_g, d, kWave);
            const int32_t ov = __shfl_xor(best_v, d, kWave), ot = __shfl_xor(best_t, d, kWave);
            if (og > best_g || (og == best_g && (ov < best_v || (ov == best_v && ot < best_t)))) {
                best_g = og;
                best_v = ov;
                best_t = ot;
            }
        }
        if (lane == 0) {
            bg[w] = best_g;
            bv[w] = best_v;
            bt[w] = best_t;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t g = bg[0];
            int32_t v = bv[0], t = bt[0];
            for (int i = 1; i < NW; i++)
                if (bg[i] > g || (bg[i] == g && (bv[i] < v || (bv[i] == v && bt[i] < t)))) {
                    g = bg[i];
                    v = bv[i];
                    t = bt[i];
                }
            if (v == INT_MAX) {
                s_over = -1;
            } else {
                const int64_t cv = vw(vwgt, v0 + v);
                const int32_t pv = lab[v0 + v] - l0;
                B[pv] -= cv;
                B[t] += cv;
                lab[v0 + v] = l0 + t;
                s_over = 1;
            }
        }
        __syncthreads();
        if (s_over < 0) {
            if (threadIdx.x == 0) balanced[blockIdx.x] = 0;
            return;
        }
    }
}

// cut of every (try, graph): cuts[try * G + graph]; one wave per vertex copy,
// lanes over its edges (the coarsest graph can hold rows of many thousands)
__global__ __launch_bounds__(256) void k_copy_cut(int32_t n, int32_t attempts, int32_t G, const int32_t *gid,
                                                  const int32_t *uxadj, const int32_t *uadj, const int32_t *uw,
                                                  const int32_t *ulab, unsigned long long *cuts) {
    const int64_t NV = (int64_t)n * attempts;
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < NV; i += waves) {
        int64_t s = 0;
        const int32_t L = ulab[i];
        const int32_t e1 = uxadj[i + 1];
        for (int32_t e = uxadj[i] + lane; e < e1; e += kWave)
            if (ulab[uadj[e]] != L) s += uw ? uw[e] : 1;
        s = wave_sum(s);
        if (lane == 0 && s) atomicAdd(&cuts[(i / n) * G + gid[i % n]], (unsigned long long)s);
    }
}

// best plain try per graph by (imbalanced, cut, try index); with an extra
// proposal (try index `attempts`), it replaces the best plain try iff it is
// balanced and the plain one is not, or it cuts no more edge weight.
__global__ void k_pick_tries(int32_t G, int32_t attempts, bool has_extra, const unsigned long long *cuts,
                             const int32_t *balanced, int32_t *chosen, int32_t *best_plain) {
    for (int32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
        int32_t b = 0;
        for (int a = 1; a < attempts; a++) {
            const int64_t ia = (int64_t)a * G + g, ib = (int64_t)b * G + g;
            const bool better = (balanced[ia] && !balanced[ib]) || (balanced[ia] == balanced[ib] && cuts[ia] < cuts[ib]);
            if (better) b = a;
        }
        best_plain[g] = b;
        if (has_extra) {
            const int64_t ie = (int64_t)attempts * G + g, ib = (int64_t)b * G + g;
            if (balanced[ie] && (!balanced[ib] || cuts[ie] <= cuts[ib])) b = attempts;
        }
        chosen[g] = b;
    }
}

// the extra proposal becomes try `attempts`: global block ids kbase[q] + b
__global__ void k_inject(int32_t n, int32_t attempts, const int32_t *xadj, bool skip_isolated, const int32_t *gid,
                         const int32_t *kbase, const int32_t *extra, int32_t *blk) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        blk[(int64_t)attempts * n + v] =
            (skip_isolated && xadj[v + 1] == xadj[v]) ? -1 : kbase[gid[v]] + extra[v];
}

__global__ void k_pick_write(int32_t n, int32_t ktot, const int32_t *gid, const int32_t *chosen, const int32_t *ulab,
                             int32_t *part) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = chosen[gid[v]];
        const int32_t L = ulab[(int64_t)b * n + v];
        part[v] = L >= 0 ? L - b * ktot : -1;
    }
}

// out[v] = q with first[q] <= v < first[q+1] (binary search per vertex)
__global__ void k_fill_range(int32_t *out, const int32_t *first, int32_t G) {
    const int32_t n = first[G];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = G - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (first[mid] <= v) lo = mid;
            else hi = mid - 1;
        }
        out[v] = lo;
    }
}

// ---------------------------------------------------------------- isolated fill

struct IsoFlag {
    const int32_t *xadj;
    __device__ bool operator()(int64_t v) const { return xadj[v + 1] == xadj[v]; }
};
struct IsoEmit {
    int32_t *iso;
    __device__ void operator()(int64_t v, int32_t pos) const { iso[pos] = (int32_t)v; }
};

__global__ void k_iso_minmax(const int32_t *iso, const int32_t *niso, const int32_t *vwgt, int32_t *mm) {
    const int32_t m = *niso;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = vwgt[iso[i]];
        atomicMin(&mm[0], c);
        atomicMax(&mm[1], c);
    }
}

// Equal weights c: the greedy "lightest block, ties lowest id" sequence equals
// the sorted merge of the sequences (B_b + j c, b), j >= 0. The i-th isolated
// vertex takes the i-th smallest element: binary search its value x, then the
// rank among blocks that reach exactly x.
//
// Past the heaviest block M = max B_b every block has one element in each
// span [M + s c, M + (s + 1) c), ordered by ((B_b - M) mod c, b); so element
// i >= T (T = number of elements below M) is block perm[(i - T) mod k], with
// perm the blocks in that order (k_iso_plan). Only i < T needs the search.
__global__ void k_iso_plan(const int64_t *B, int32_t k, int64_t c, int64_t *MT, int32_t *perm) {
    __shared__ int64_t sM;
    if (threadIdx.x == 0) {
        int64_t M = LLONG_MIN;
        for (int b = 0; b < k; b++) M = B[b] > M ? B[b] : M;
        int64_t T = 0;
        for (int b = 0; b < k; b++) T += (M - B[b] + c - 1) / c;
        MT[0] = M;
        MT[1] = T;
        sM = M;
    }
    __syncthreads();
    const int64_t M = sM;
    for (int b = threadIdx.x; b < k; b += blockDim.x) {
        const int64_t ob = ((B[b] - M) % c + c) % c;
        int32_t rank = 0;
        for (int q = 0; q < k; q++) {
            const int64_t oq = ((B[q] - M) % c + c) % c;
            rank += oq < ob || (oq == ob && q < b);
        }
        perm[rank] = b;
    }
}

// UNIT: every isolated vertex weighs 1 (c == 1), so the divisions by c drop out
template <bool UNIT>
__global__ void k_iso_uniform(const int32_t *iso, const int32_t *niso, const int64_t *B, int32_t k, int64_t c,
                              const int64_t *MT, const int32_t *perm, int32_t *part) {
    const int32_t m = *niso;
    const int64_t T = MT[1];
    int64_t bmin = LLONG_MAX;
    for (int b = 0; b < k; b++) bmin = B[b] < bmin ? B[b] : bmin;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        if (i >= T) {
            part[iso[i]] = perm[(i - T) % k];
            continue;
        }
        // f(x) = #elements <= x
        int64_t lo = bmin, hi = bmin + i * c;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            int64_t f = 0;
            for (int b = 0; b < k; b++)
                if (B[b] <= mid) f += (UNIT ? (mid - B[b]) : (mid - B[b]) / c) + 1;
            if (f >= i + 1) hi = mid;
            else lo = mid + 1;
        }
        const int64_t x = lo;
        int64_t below = 0;  // elements < x
        for (int b = 0; b < k; b++)
            if (B[b] <= x - 1) below += (UNIT ? (x - 1 - B[b]) : (x - 1 - B[b]) / c) + 1;
        int64_t rank = i - below;
        int32_t pick = -1;
        for (int b = 0; b < k; b++) {
            if (B[b] <= x && (UNIT || (x - B[b]) % c == 0)) {
                if (rank == 0) {
                    pick = b;
                    break;
                }
                rank--;
            }
        }
        part[iso[i]] = pick;
    }
}

// General weights: one thread, binary heap of (B_b, b).
__global__ void k_iso_serial(const int32_t *iso, const int32_t *niso, const int64_t *B0, int32_t k,
                             const int32_t *vwgt, int64_t *hv, int32_t *hb, int32_t *part) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    auto less = [&](int i, int j) { return hv[i] < hv[j] || (hv[i] == hv[j] && hb[i] < hb[j]); };
    for (int b = 0; b < k; b++) {
        hv[b] = B0[b];
        hb[b] = b;
        int i = b;
        while (i > 0) {
            int p = (i - 1) / 2;
            if (!less(i, p)) break;
            int64_t tv = hv[i];
            hv[i] = hv[p];
            hv[p] = tv;
            int32_t tb = hb[i];
            hb[i] = hb[p];
            hb[p] = tb;
            i = p;
        }
    }
    const int32_t m = *niso;
    for (int32_t q = 0; q < m; q++) {
        const int32_t v = iso[q];
        part[v] = hb[0];
        hv[0] += vwgt ? vwgt[v] : 1;
        int i = 0;
        for (;;) {
            int l = 2 * i + 1, r = l + 1, s = i;
            if (l < k && less(l, s)) s = l;
            if (r < k && less(r, s)) s = r;
            if (s == i) break;
            int64_t tv = hv[i];
            hv[i] = hv[s];
            hv[s] = tv;
            int32_t tb = hb[i];
            hb[i] = hb[s];
            hb[s] = tb;
            i = s;
        }
    }
}

// Batched placement of vertices without neighbours. The list iso[] is in
// ascending id, hence grouped by graph; vertex iso[i] belongs to graph
// q = gid[iso[i]] and is the (i - iso_first[q])-th of its graph.
template <bool UNIT>
__global__ void k_iso_uniform_batch(const int32_t *iso, const int32_t *niso, const int32_t *gid,
                                    const int32_t *iso_first, const int32_t *kbase, const int64_t *Ball, int64_t c,
                                    int32_t *part) {
    const int32_t m = *niso;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = gid[iso[i]];
        const int64_t r = i - iso_first[q];
        const int32_t k = kbase[q + 1] - kbase[q];
        const int64_t *B = Ball + kbase[q];
        int64_t bmin = LLONG_MAX;
        for (int b = 0; b < k; b++) bmin = B[b] < bmin ? B[b] : bmin;
        int64_t lo = bmin, hi = bmin + r * c;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            int64_t f = 0;
            for (int b = 0; b < k; b++)
                if (B[b] <= mid) f += (UNIT ? (mid - B[b]) : (mid - B[b]) / c) + 1;
            if (f >= r + 1) hi = mid;
            else lo = mid + 1;
        }
        const int64_t x = lo;
        int64_t below = 0;
        for (int b = 0; b < k; b++)
            if (B[b] <= x - 1) below += (UNIT ? (x - 1 - B[b]) : (x - 1 - B[b]) / c) + 1;
        int64_t rank = r - below;
        int32_t pick = -1;
        for (int b = 0; b < k; b++) {
            if (B[b] <= x && (UNIT || (x - B[b]) % c == 0)) {
                if (rank == 0) {
                    pick = b;
                    break;
                }
                rank--;
            }
        }
        part[iso[i]] = pick >= 0 ? kbase[q] + pick : -1;
    }
}

// General weights: one thread per graph, binary heap of (B_b, b) in hv/hb at kbase[q].
__global__ void k_iso_serial_batch(const int32_t *iso, const int32_t *iso_first, int32_t G, const int32_t *kbase,
                                   const int64_t *Ball, const int32_t *vwgt, int64_t *hvall, int32_t *hball,
                                   int32_t *part) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < G; q += gridDim.x * blockDim.x) {
        const int32_t k = kbase[q + 1] - kbase[q];
        int64_t *hv = hvall + kbase[q];
        int32_t *hb = hball + kbase[q];
        auto less = [&](int i, int j) { return hv[i] < hv[j] || (hv[i] == hv[j] && hb[i] < hb[j]); };
        for (int b = 0; b < k; b++) {
            hv[b] = Ball[kbase[q] + b];
            hb[b] = b;
            int i = b;
            while (i > 0) {
                const int p = (i - 1) / 2;
                if (!less(i, p)) break;
                const int64_t tv = hv[i];
                hv[i] = hv[p];
                hv[p] = tv;
                const int32_t tb = hb[i];
                hb[i] = hb[p];
                hb[p] = tb;
                i = p;
            }
        }
        for (int32_t x = iso_first[q]; x < iso_first[q + 1]; x++) {
            const int32_t v = iso[x];
            part[v] = kbase[q] + hb[0];
            hv[0] += vwgt ? vwgt[v] : 1;
            int i = 0;
            for (;;) {
                const int l = 2 * i + 1, r = l + 1;
                int sm = i;
                if (l < k && less(l, sm)) sm = l;
                if (r < k && less(r, sm)) sm = r;
                if (sm == i) break;
                const int64_t tv = hv[i];
                hv[i] = hv[sm];
                hv[sm] = tv;
                const int32_t tb = hb[i];
                hb[i] = hb[sm];
                hb[sm] = tb;
                i = sm;
            }
        }
    }
}

}  // namespace

int initial_partition_batch(const DevGraph &g, bool skip_isolated, const BatchInfo &bi, uint64_t seed,
                            int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, int32_t fm_passes,
                            bool wide, int32_t *part, Scratch &sc, const int32_t *extra, ProposalOut *po) {
    ScratchScope scope(sc);  // part and po are the outputs: all scratch below is internal
    hipStream_t s = sc.stream();
    const int32_t n = g.n, nnz = g.nnz, G = bi.G;
    if (n == 0) return GP_OK;
    const int32_t bis = attempts;             // bisection tries
    if (extra) attempts += 1;                 // the proposal is one more try
    const int32_t ktot = bi.kbase[G];
    int32_t kmax = 1;
    for (int32_t q = 0; q < G; q++) kmax = std::max(kmax, bi.k[q]);
    if ((int64_t)n * attempts >= INT_MAX || (int64_t)nnz * attempts >= INT_MAX ||
        (int64_t)ktot * attempts >= INT_MAX) {
        set_error("initial partition: coarsest graph times attempts exceeds int32 indexing");
        return GP_ERR_OVERFLOW;
    }
    if (kmax > 2048) {
        set_error("initial partition: k > 2048 is not supported by the rebalance kernel");
        return GP_ERR_ARG;
    }
    // ---- recursion trees of (graph, local base, k_S) per depth (each depends only on k_g)
    std::vector<std::vector<std::array<int32_t, 3>>> depth;
    for (int32_t q = 0; q < G; q++) {
        std::vector<std::pair<int32_t, int32_t>> cur{{0, bi.k[q]}};
        for (size_t d = 0; !cur.empty(); d++) {
            std::vector<std::pair<int32_t, int32_t>> next;
            for (auto &p : cur)
                if (p.second > 1) {
                    if (depth.size() <= d) depth.resize(d + 1);
                    depth[d].push_back({q, p.first, p.second});
                    const int32_t kl = (p.second + 1) / 2;
                    next.push_back({p.first, kl});
                    next.push_back({p.first + kl, p.second - kl});
                }
            cur = next;
        }
    }
    // per-workgroup regions sized by the subproblem's graph
    int64_t regmax = 1;
    size_t maxsub = 1;
    for (auto &d : depth) {
        int64_t t = 0;
        for (auto &e : d) t += bi.voff[e[0] + 1] - bi.voff[e[0]];
        regmax = std::max(regmax, t);
        maxsub = std::max(maxsub, d.size());
    }
    int32_t *blk = nullptr, *mark = nullptr, *claim = nullptr, *slist = nullptr, *order = nullptr, *pre = nullptr,
            *sg = nullptr, *sb = nullptr, *sk = nullptr;
    int64_t *reg = nullptr;
    GP_TRY(sc.alloc(&blk, (size_t)n * attempts));
    GP_TRY(sc.alloc(&mark, (size_t)n * attempts));
    GP_TRY(sc.alloc(&claim, (size_t)n * attempts));
    GP_TRY(sc.alloc(&slist, (size_t)regmax * attempts));
    GP_TRY(sc.alloc(&order, (size_t)regmax * attempts));
    GP_TRY(sc.alloc(&pre, (size_t)(regmax + maxsub) * attempts));
    GP_TRY(sc.alloc(&sg, maxsub));
    GP_TRY(sc.alloc(&sb, maxsub));
    GP_TRY(sc.alloc(&sk, maxsub));
    GP_TRY(sc.alloc(&reg, maxsub));
    int64_t *gain = nullptr;
    if (fm_passes > 0) GP_TRY(sc.alloc(&gain, (size_t)n * attempts));
    hipLaunchKernelGGL(k_init_blk, dim3(grid_for((int64_t)n * attempts, 256, 65536)), dim3(256), 0, s, n, attempts,
                       g.xadj, skip_isolated, bi.d_gid, bi.d_kbase, blk);
    GP_LAUNCH_CHECK();
    std::vector<int32_t> hg, hb, hk;
    std::vector<int64_t> hr;
    for (auto &d : depth) {
        hg.clear();
        hb.clear();
        hk.clear();
        hr.clear();
        int64_t off = 0;
        for (auto &e : d) {
            hg.push_back(e[0]);
            hb.push_back(e[1]);
            hk.push_back(e[2]);
            hr.push_back(off);
            off += bi.voff[e[0] + 1] - bi.voff[e[0]];
        }
        GP_HIP(hipMemcpyAsync(sg, hg.data(), sizeof(int32_t) * hg.size(), hipMemcpyHostToDevice, s));
        GP_HIP(hipMemcpyAsync(sb, hb.data(), sizeof(int32_t) * hb.size(), hipMemcpyHostToDevice, s));
        GP_HIP(hipMemcpyAsync(sk, hk.data(), sizeof(int32_t) * hk.size(), hipMemcpyHostToDevice, s));
        GP_HIP(hipMemcpyAsync(reg, hr.data(), sizeof(int64_t) * hr.size(), hipMemcpyHostToDevice, s));
        BisectArgs a{n,    g.xadj, g.adjncy, g.vwgt, blk,        mark,       claim,           slist,
                     order, pre,   reg,      off,    sg,   sb, sk, bi.d_voff, bi.d_kbase, (int32_t)d.size(), seed};
        hipLaunchKernelGGL(k_bisect, dim3((unsigned)(d.size() * bis)), dim3(kBB), 0, s, a);
        GP_LAUNCH_CHECK();
        if (fm_passes > 0) {
            FmArgs fa{g.xadj, g.adjncy, g.adjwgt, g.vwgt, n,   blk,        mark,       gain,
                      claim,  slist,    order,    reg,     off,    sg,  sb,         sk,
                      bi.d_voff, bi.d_kbase, bi.d_lmax, (int32_t)d.size(), fm_passes, (int32_t)wide};
            hipLaunchKernelGGL(k_fm, dim3((unsigned)(d.size() * bis)), dim3(kBB), 0, s, fa);
            GP_LAUNCH_CHECK();
        }
        // host vectors are reused next depth: make sure the copies have been consumed
        GP_HIP(hipStreamSynchronize(s));
    }
    if (extra) {
        hipLaunchKernelGGL(k_inject, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, bis, g.xadj, skip_isolated,
                           bi.d_gid, bi.d_kbase, extra, blk);
        GP_LAUNCH_CHECK();
    }

    // ---- refine all tries of all graphs at once on the disjoint union
    const int32_t NV = n * attempts, NE = nnz * attempts;
    int32_t *ux = nullptr, *ua = nullptr, *uw = nullptr, *uv = nullptr, *ul = nullptr;
    GP_TRY(sc.alloc(&ux, (size_t)NV + 1));
    GP_TRY(sc.alloc(&ua, NE));
    if (g.adjwgt) GP_TRY(sc.alloc(&uw, NE));
    if (g.vwgt) GP_TRY(sc.alloc(&uv, NV));
    GP_TRY(sc.alloc(&ul, NV));
    hipLaunchKernelGGL(k_union, dim3(grid_for((int64_t)NE + NV, 256, 65536)), dim3(256), 0, s, n, nnz, attempts, ktot,
                       g.xadj, g.adjncy, g.adjwgt, g.vwgt, blk, ux, ua, uw, uv, ul);
    GP_LAUNCH_CHECK();
    DevGraph ug;
    ug.n = NV;
    ug.nnz = NE;
    ug.xadj = ux;
    ug.adjncy = ua;
    ug.adjwgt = uw;
    ug.vwgt = uv;
    const int32_t NL = ktot * attempts;
    int64_t *W = nullptr, *cap = nullptr;
    GP_TRY(sc.alloc(&W, NL));
    GP_TRY(label_weights(ug, ul, W, NL, sc));
    if (G > 1) {
        GP_TRY(sc.alloc(&cap, NL));
        hipLaunchKernelGGL(k_label_caps, dim3(grid_for(NL, 256, 4096)), dim3(256), 0, s, attempts, ktot, G,
                           bi.d_kbase, bi.d_lmax, cap);
        GP_LAUNCH_CHECK();
    }
    GP_TRY(lp_run(ug, ul, W, NL, bi.lmax[0], rounds_refine, dir_alternate, wide, nullptr, sc, cap));

    // ---- rebalance each (try, graph), pick the best try per graph
    int32_t *bal = nullptr, *ch = nullptr, *bp = nullptr;
    unsigned long long *cuts = nullptr;
    const int64_t TG = (int64_t)attempts * G;
    GP_TRY(sc.alloc(&bal, TG));
    GP_TRY(sc.alloc(&cuts, TG));
    GP_TRY(sc.alloc(&ch, G));
    GP_TRY(sc.alloc(&bp, G));
    GP_HIP(hipMemsetAsync(cuts, 0, sizeof(unsigned long long) * TG, s));
    const size_t dyn = sizeof(int64_t) * (size_t)kmax * (1 + kRB / kWave);
    GP_HIP(hipFuncSetAttribute((const void *)k_rebalance, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    hipLaunchKernelGGL(k_rebalance, dim3((unsigned)TG), dim3(kRB), dyn, s, n, G, ktot, bi.d_voff, bi.d_kbase,
                       bi.d_lmax, ux, ua, uw, uv, ul, bal, kmax);
    GP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_copy_cut, dim3(grid_for(NV, 4, 65536)), dim3(256), 0, s, n, attempts, G, bi.d_gid, ux, ua,
                       uw, ul, cuts);
    GP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pick_tries, dim3(grid_for(G, 256, 1024)), dim3(256), 0, s, G, bis, extra != nullptr, cuts,
                       bal, ch, bp);
    hipLaunchKernelGGL(k_pick_write, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, ktot, bi.d_gid, ch, ul, part);
    GP_LAUNCH_CHECK();
    if (extra && po) {
        std::vector<unsigned long long> hc(TG);
        std::vector<int32_t> hch(G), hbp(G);
        GP_HIP(hipMemcpyAsync(hc.data(), cuts, sizeof(unsigned long long) * TG, hipMemcpyDeviceToHost, s));
        GP_HIP(hipMemcpyAsync(hch.data(), ch, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
        GP_HIP(hipMemcpyAsync(hbp.data(), bp, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        po->plain_cut.resize(G);
        po->prop_cut.resize(G);
        po->kept.resize(G);
        for (int32_t q = 0; q < G; q++) {  // k_copy_cut counts each edge from both ends
            po->plain_cut[q] = (int64_t)(hc[(size_t)hbp[q] * G + q] / 2);
            po->prop_cut[q] = (int64_t)(hc[(size_t)bis * G + q] / 2);
            po->kept[q] = hch[q] == bis;
        }
    }
    return GP_OK;
}

int graph_ids(int32_t G, int32_t n, const int32_t *d_voff, int32_t *gid, hipStream_t s) {
    if (n <= 0) return GP_OK;
    hipLaunchKernelGGL(k_fill_range, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, gid, d_voff, G);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

int initial_partition(const DevGraph &g, bool skip_isolated, int32_t k, int64_t lmax, uint64_t seed,
                      int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, int32_t fm_passes, bool wide,
                      int32_t *part, Scratch &sc, const int32_t *extra, ProposalOut *po) {
    if (g.n == 0) return GP_OK;
    BatchInfo bi;
    bi.G = 1;
    bi.voff = {0, g.n};
    bi.k = {k};
    bi.kbase = {0, k};
    bi.lmax = {lmax};
    int32_t *dv = nullptr, *dk = nullptr, *gid = nullptr;
    int64_t *dl = nullptr;
    GP_TRY(sc.alloc(&dv, 2));
    GP_TRY(sc.alloc(&dk, 2));
    GP_TRY(sc.alloc(&dl, 1));
    GP_TRY(sc.alloc(&gid, g.n));
    GP_HIP(hipMemcpyAsync(dv, bi.voff.data(), sizeof(int32_t) * 2, hipMemcpyHostToDevice, sc.stream()));
    GP_HIP(hipMemcpyAsync(dk, bi.kbase.data(), sizeof(int32_t) * 2, hipMemcpyHostToDevice, sc.stream()));
    GP_HIP(hipMemcpyAsync(dl, bi.lmax.data(), sizeof(int64_t), hipMemcpyHostToDevice, sc.stream()));
    GP_HIP(hipMemsetAsync(gid, 0, sizeof(int32_t) * (size_t)g.n, sc.stream()));
    bi.d_voff = dv;
    bi.d_kbase = dk;
    bi.d_lmax = dl;
    bi.d_gid = gid;
    return initial_partition_batch(g, skip_isolated, bi, seed, attempts, rounds_refine, dir_alternate, fm_passes,
                                   wide, part, sc, extra, po);
}

int fill_isolated(const DevGraph &g, int32_t k, int32_t *part, const int64_t *B, int32_t *niso_host, Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = g.n;
    int32_t *iso = nullptr, *d_niso = nullptr, *mm = nullptr;
    GP_TRY(sc.alloc(&iso, n));
    GP_TRY(sc.alloc(&d_niso, 1));
    GP_TRY(sc.alloc(&mm, 2));
    GP_TRY(compact(IsoFlag{g.xadj}, IsoEmit{iso}, n, nullptr, d_niso, sc));
    int32_t h[2] = {1, 1}, niso = 0;
    GP_HIP(hipMemcpyAsync(&niso, d_niso, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (g.vwgt) {
        const int32_t init[2] = {INT_MAX, INT_MIN};
        GP_HIP(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_iso_minmax, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, iso, d_niso, g.vwgt, mm);
        GP_LAUNCH_CHECK();
        GP_HIP(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, s));
    }
    GP_HIP(hipStreamSynchronize(s));
    if (niso_host) *niso_host = niso;
    if (niso == 0) return GP_OK;
    if (h[0] == h[1]) {
        int64_t *MT = nullptr;
        int32_t *perm = nullptr;
        GP_TRY(sc.alloc(&MT, 2));
        GP_TRY(sc.alloc(&perm, k));
        hipLaunchKernelGGL(k_iso_plan, dim3(1), dim3(256), 0, s, B, k, (int64_t)h[0], MT, perm);
        if (h[0] == 1)
            hipLaunchKernelGGL(k_iso_uniform<true>, dim3(grid_for(niso, 256, 8192)), dim3(256), 0, s, iso, d_niso, B,
                               k, (int64_t)1, MT, perm, part);
        else
            hipLaunchKernelGGL(k_iso_uniform<false>, dim3(grid_for(niso, 256, 8192)), dim3(256), 0, s, iso, d_niso, B,
                               k, (int64_t)h[0], MT, perm, part);
        GP_LAUNCH_CHECK();
    } else {
        int64_t *hv = nullptr;
        int32_t *hbk = nullptr;
        GP_TRY(sc.alloc(&hv, k));
        GP_TRY(sc.alloc(&hbk, k));
        hipLaunchKernelGGL(k_iso_serial, dim3(1), dim3(64), 0, s, iso, d_niso, B, k, g.vwgt, hv, hbk, part);
        GP_LAUNCH_CHECK();
    }
    return GP_OK;
}

}  // namespace gp

namespace gp {

int fill_isolated_batch(const DevGraph &g, const BatchInfo &bi, const int32_t *d_iso_first, int32_t *part,
                        const int64_t *B, Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = g.n;
    if (n == 0) return GP_OK;
    int32_t *iso = nullptr, *d_niso = nullptr, *mm = nullptr;
    GP_TRY(sc.alloc(&iso, n));
    GP_TRY(sc.alloc(&d_niso, 1));
    GP_TRY(sc.alloc(&mm, 2));
    GP_TRY(compact(IsoFlag{g.xadj}, IsoEmit{iso}, n, nullptr, d_niso, sc));
    int32_t h[2] = {1, 1}, niso = 0;
    GP_HIP(hipMemcpyAsync(&niso, d_niso, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (g.vwgt) {
        const int32_t init[2] = {INT_MAX, INT_MIN};
        GP_HIP(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_iso_minmax, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, iso, d_niso, g.vwgt, mm);
        GP_LAUNCH_CHECK();
        GP_HIP(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, s));
    }
    GP_HIP(hipStreamSynchronize(s));
    if (niso == 0) return GP_OK;
    if (h[0] == h[1]) {
        if (h[0] == 1)
            hipLaunchKernelGGL(k_iso_uniform_batch<true>, dim3(grid_for(niso, 256, 8192)), dim3(256), 0, s, iso,
                               d_niso, bi.d_gid, d_iso_first, bi.d_kbase, B, (int64_t)1, part);
        else
            hipLaunchKernelGGL(k_iso_uniform_batch<false>, dim3(grid_for(niso, 256, 8192)), dim3(256), 0, s, iso,
                               d_niso, bi.d_gid, d_iso_first, bi.d_kbase, B, (int64_t)h[0], part);
        GP_LAUNCH_CHECK();
    } else {
        int64_t *hv = nullptr;
        int32_t *hb = nullptr;
        GP_TRY(sc.alloc(&hv, bi.kbase[bi.G]));
        GP_TRY(sc.alloc(&hb, bi.kbase[bi.G]));
        hipLaunchKernelGGL(k_iso_serial_batch, dim3(grid_for(bi.G, 64, 4096)), dim3(64), 0, s, iso, d_iso_first, bi.G,
                           bi.d_kbase, B, g.vwgt, hv, hb, part);
        GP_LAUNCH_CHECK();
    }
    return GP_OK;
}

}  // namespace gp
