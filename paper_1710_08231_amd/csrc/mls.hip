// mls.hip — multi-try k-way local search (MLS, §III-C) on gfx950, in the
// data-parallel form of the paper's parallel MLS (§IV-C, Algorithm 1 with
// PerformMoves and ApplyMoves).
//
// The paper's PEs run searches concurrently on a partition that stays fixed
// for a local iteration, keep their moves private, and ApplyMoves replays
// each PE's moves with recomputed gains so that L_max is never broken. Here
// the interleaving is fixed so that results are deterministic:
//  - a batch takes the next seeds of the todo order (skipping vertices marked
//    at the batch's start) while their closed neighbourhoods are pairwise
//    disjoint, at most `batch` of them;
//  - every search of the batch runs on one wavefront from the batch's
//    partition, block weights and marks, seeing none of its batch-mates'
//    moves or marks: its queued vertices (at most `queue`, one per lane),
//    their gains, its private labels and block weights live in LDS;
//  - one workgroup then applies the kept prefixes in seed order, recomputing
//    every gain on the current partition (ApplyMoves), and the union of the
//    batch's marks holds for the rest of the local iteration.
//
// Per search (§III-C): queue the seed and its unmarked neighbours; repeatedly
// take the queued vertex of largest gain (ties: lower id), re-queue it with
// its current gain if that changed, otherwise move it to its best block,
// then re-evaluate queued neighbours and queue unmarked ones; stop when the
// queue is empty or after max_idle moves without a new best; keep the
// shortest prefix of largest positive cumulative gain. gain(v) is the
// largest connection to an adjacent other block with room for v under L_max
// (ties: lowest block) minus the connection to v's own block.
#include <climits>

#include "mls.hpp"
#include "prims.hpp"

namespace gp {
namespace {

constexpr int kHT = 128;      // per-search hash of queued vertices (slots; at most 64 keys)
constexpr int kSW = 4;        // searches (wavefronts) per workgroup
constexpr int kAB = 1024;     // threads of the single-workgroup kernels
constexpr int kGG = 8;        // flagged queue entries whose gains one edge pass evaluates together

struct Ctl {
    int32_t ti, ntodo, nsel, tiw;  // todo cursor, todo length, window seeds, todo index after the window
    int32_t clash;                 // first window index whose closed neighbourhood meets an earlier one's
    uint32_t epoch;                // batch number; claims of earlier batches read as empty
    int32_t nnext, nmark;          // moved vertices of the local iteration, marked vertices
    long long lgain, kept, searches;
};

struct MG {
    const int32_t *xadj, *adjncy, *adjwgt, *vwgt;
};

__device__ __forceinline__ long long vw(const MG &g, int32_t v) { return g.vwgt ? g.vwgt[v] : 1; }
__device__ __forceinline__ long long ew(const MG &g, int32_t e) { return g.adjwgt ? g.adjwgt[e] : 1; }

__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // splitmix64 finaliser of x + golden gamma
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// ---------------------------------------------------------------- per global / local iteration

__global__ void k_boundary(MG g, const int32_t *part, int32_t n, int32_t *flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = part[v];
        int32_t b = 0;
        for (int32_t e = g.xadj[v]; e < g.xadj[v + 1] && !b; e++) b = part[g.adjncy[e]] != p;
        flag[v] = p >= 0 && b;
    }
}

struct FlagSet {
    const int32_t *flag;
    __device__ bool operator()(int64_t i) const { return flag[i] != 0; }
};
struct EmitId {
    int32_t *out;
    __device__ void operator()(int64_t i, int32_t pos) const { out[pos] = (int32_t)i; }
};

// keys of the hash order: mix64(h ^ id(v)) (distinct for distinct ids: mix64 is a bijection)
__global__ void k_order_keys(const int32_t *todo, const Ctl *c, const int32_t *hash_id, uint64_t h, uint64_t *key) {
    const int32_t nt = c->ntodo;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = todo[i];
        key[i] = mix64(h ^ (uint64_t)(uint32_t)(hash_id ? hash_id[v] : v));
    }
}

__global__ void k_begin_global(Ctl *c, const int32_t *count) {
    c->ntodo = *count;
    c->nnext = 0;
}

__global__ void k_begin_local(Ctl *c) {
    c->ti = 0;
    c->nnext = 0;
    c->lgain = 0;
}

__global__ void k_next_to_todo(const int32_t *next, int32_t *todo, Ctl *c) {
    const int32_t nn = c->nnext;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (int64_t)gridDim.x * blockDim.x)
        todo[i] = next[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) c->ntodo = nn;
}

__global__ void k_unmark(int32_t *marked, const int32_t *marklist, Ctl *c) {
    const int32_t nm = c->nmark;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nm; i += (int64_t)gridDim.x * blockDim.x)
        marked[marklist[i]] = 0;
}

__global__ void k_reset_marks(Ctl *c) { c->nmark = 0; }

// ---------------------------------------------------------------- one batch

// The next seeds: unmarked todo entries from the cursor, at most `batch`.
__global__ __launch_bounds__(kAB) void k_window(const int32_t *todo, const int32_t *marked, int32_t batch, Ctl *c,
                                                int32_t *sel, int32_t *selpos) {
    __shared__ int32_t tmp[kAB / kWave + 1];
    __shared__ int32_t s_sel, s_end;
    const int32_t ti = c->ti, ntodo = c->ntodo;
    if (threadIdx.x == 0) {
        s_sel = 0;
        s_end = ntodo;
    }
    __syncthreads();
    for (int32_t p0 = ti; p0 < ntodo; p0 += kAB) {
        const int32_t base = s_sel;
        const int32_t idx = p0 + (int32_t)threadIdx.x;
        const int32_t f = (idx < ntodo && !marked[todo[idx]]) ? 1 : 0;
        int32_t tot = 0;
        const int32_t r = block_excl_scan<kAB, int32_t>(f, tmp, &tot);
        if (f && base + r < batch) {
            sel[base + r] = todo[idx];
            selpos[base + r] = idx;
            if (base + r == batch - 1) s_end = idx + 1;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_sel = min(batch, base + tot);
        __syncthreads();
        if (s_sel >= batch) break;
    }
    if (threadIdx.x == 0) {
        c->nsel = s_sel;
        c->tiw = s_end;
        c->clash = INT_MAX;
    }
}

// Claims of the window seeds' closed neighbourhoods. first[u] keeps the
// smallest claimant of this batch tagged with the batch number (a newer batch
// has a smaller tag, so it always overwrites older claims). Whichever of the
// two smallest claimants of u comes second sees the other and offers the
// larger index, i.e. u's second-smallest claimant; the smallest offer over
// all u is the first seed whose neighbourhood meets an earlier one's.
__global__ __launch_bounds__(256) void k_claim(MG g, const int32_t *sel, Ctl *c, unsigned long long *first) {
    const int32_t i = blockIdx.x;
    if (i >= c->nsel) return;
    const int32_t s = sel[i];
    const uint32_t tag = ~c->epoch;
    const int32_t b = g.xadj[s], e = g.xadj[s + 1];
    for (int32_t t = b - 1 + (int32_t)threadIdx.x; t < e; t += blockDim.x) {
        const int32_t u = t < b ? s : g.adjncy[t];
        const unsigned long long old = atomicMin(&first[u], ((unsigned long long)tag << 32) | (uint32_t)i);
        if ((uint32_t)(old >> 32) == tag) atomicMin(&c->clash, max((int32_t)(uint32_t)old, i));
    }
}

struct SearchArgs {
    MG g;
    int32_t k;
    int64_t lmax;
    const int32_t *part;
    const int64_t *B;
    const int32_t *marked;
    const int32_t *sel;
    const Ctl *c;
    int32_t q, max_idle;
    int32_t *mv_v, *mv_f, *mv_t, *mv_n;  // kept prefix of search j at j * kMlsMaxQueue
    int32_t *mk_v, *mk_n;                // vertices search j queued (its marks)
};

struct WaveLds {
    long long conn[kGG][kMlsMaxK];  // connection sums of the vertices being evaluated
    int32_t gpre[kGG + 1], gbase[kGG], gslot[kGG];  // a group of evaluations: edge prefix, row start, slot
    long long Bp[kMlsMaxK];    // the search's block weights
    long long key[kMlsMaxQueue];
    int32_t hk[kHT], hs[kHT];  // queued vertex -> slot
    int32_t qv[kMlsMaxQueue];   // queued vertices, in queueing order
    int32_t plab[kMlsMaxQueue]; // their labels in the search's view
    int32_t inh[kMlsMaxQueue];  // in the queue
    int32_t flag[kMlsMaxQueue]; // 1: re-evaluate, 2: newly queued
    int32_t lv[kMlsMaxQueue], lf[kMlsMaxQueue], lt[kMlsMaxQueue];  // move log
};

__device__ __forceinline__ uint32_t hslot(int32_t x) { return ((uint32_t)x * 0x9E3779B1u) >> (32 - 7); }

__device__ __forceinline__ int32_t h_find(const WaveLds &L, int32_t x) {
    uint32_t h = hslot(x);
    for (;;) {
        const int32_t kx = L.hk[h];
        if (kx == x) return L.hs[h];
        if (kx < 0) return -1;
        h = (h + 1) & (kHT - 1);
    }
}

// distinct keys only; lanes may insert concurrently
__device__ __forceinline__ void h_insert(WaveLds &L, int32_t x, int32_t slot) {
    uint32_t h = hslot(x);
    for (;;) {
        if (atomicCAS(&L.hk[h], -1, x) == -1) {
            L.hs[h] = slot;
            return;
        }
        h = (h + 1) & (kHT - 1);
    }
}

__device__ __forceinline__ int32_t label_in(const SearchArgs &a, const WaveLds &L, int32_t x) {
    const int32_t s = h_find(L, x);
    return s >= 0 ? L.plab[s] : a.part[x];
}

__device__ __forceinline__ void best_pair(long long &bc, int32_t &bl) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const long long oc = __shfl_xor(bc, d, kWave);
        const int32_t ol = __shfl_xor(bl, d, kWave);
        if (oc > bc || (oc == bc && ol < bl)) {
            bc = oc;
            bl = ol;
        }
    }
}

// From a vertex's connection sums: the best adjacent other block with room
// for it under L_max (ties: lowest block) and the gain of moving there;
// target -1 when there is none. Clears the sums (wave-uniform call).
__device__ void select_gain(const SearchArgs &a, long long *conn, const long long *Bp, int32_t own, long long cu,
                            long long &gain, int32_t &target) {
    const int lane = lane_id();
    long long bc = 0;
    int32_t bl = INT_MAX;
    for (int32_t b = lane; b < a.k; b += kWave) {
        const long long cb = conn[b];
        if (b != own && cb > 0 && Bp[b] + cu <= a.lmax && (cb > bc || (cb == bc && b < bl))) {
            bc = cb;
            bl = b;
        }
    }
    best_pair(bc, bl);
    const long long oc = conn[own];
    wave_sync();
    for (int32_t b = lane; b < a.k; b += kWave) conn[b] = 0;
    wave_sync();
    target = bl == INT_MAX ? -1 : bl;
    gain = bc - oc;
}

// gain and target of the queued vertex in slot su, in the search's view;
// target -1 when no adjacent other block has room (wave-uniform call)
__device__ void wave_gain(const SearchArgs &a, WaveLds &L, int32_t su, long long &gain, int32_t &target) {
    const int lane = lane_id();
    const int32_t u = L.qv[su];
    const int32_t own = L.plab[su];
    const long long cu = vw(a.g, u);
    const int32_t b0 = a.g.xadj[u], b1 = a.g.xadj[u + 1];
    for (int32_t e = b0 + lane; e < b1; e += kWave)
        atomicAdd((unsigned long long *)&L.conn[0][label_in(a, L, a.g.adjncy[e])], (unsigned long long)ew(a.g, e));
    wave_sync();
    select_gain(a, L.conn[0], L.Bp, own, cu, gain, target);
}

// Queues, in list order, the unmarked vertices of list[0, len) (list == null:
// the vertex `self` alone) that are not queued yet, while fewer than q are
// queued; every vertex of the list already in the queue is flagged for
// re-evaluation. Returns the new queue length (wave-uniform).
__device__ int32_t scan_list(const SearchArgs &a, WaveLds &L, const int32_t *list, int32_t len, int32_t self,
                             int32_t queued) {
    const int lane = lane_id();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int32_t i0 = 0; i0 < len; i0 += kWave) {
        const int32_t i = i0 + lane;
        const int32_t x = i < len ? (list ? list[i] : self) : -1;
        const int32_t s = x >= 0 ? h_find(L, x) : -1;
        if (s >= 0 && L.inh[s]) L.flag[s] = 1;
        const bool cand = x >= 0 && s < 0 && !a.marked[x];
        const uint64_t m = __ballot(cand);
        wave_sync();
        const int32_t room = a.q - queued;
        const int32_t r = (int32_t)__popcll(m & lt);
        if (cand && r < room) {
            const int32_t slot = queued + r;
            L.qv[slot] = x;
            L.plab[slot] = a.part[x];
            L.flag[slot] = 2;
            h_insert(L, x, slot);
        }
        queued += min((int32_t)__popcll(m), room);
        wave_sync();
    }
    return queued;
}

// Evaluates the flagged slots: re-evaluated queue entries take their new gain
// (or leave the queue), newly queued vertices enter it if they have a move.
// Every gain is taken on the same state, so up to kGG of them share one pass
// over their concatenated edge lists (slot s sits on lane s).
__device__ void eval_flags(const SearchArgs &a, WaveLds &L, int32_t queued) {
    const int lane = lane_id();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    uint64_t rem = __ballot(lane < queued && L.flag[lane] != 0);
    while (rem) {
        // the next kGG flagged slots, in slot order
        uint64_t grp = rem;
        for (int i = 0, c = (int)__popcll(rem); i < c - kGG; i++) grp &= ~(1ull << (63 - __clzll(grp)));
        rem &= ~grp;
        const int ng = (int)__popcll(grp);
        const bool member = (grp >> lane) & 1ull;
        const int r = (int)__popcll(grp & lt);
        int32_t d = 0, b0 = 0;
        if (member) {
            const int32_t u = L.qv[lane];
            b0 = a.g.xadj[u];
            d = a.g.xadj[u + 1] - b0;
        }
        int32_t inc = d;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t y = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += y;
        }
        if (member) {
            L.gpre[r] = inc - d;
            L.gbase[r] = b0;
            L.gslot[r] = lane;
        }
        const int32_t total = __shfl(inc, kWave - 1, kWave);
        if (lane == 0) L.gpre[ng] = total;
        wave_sync();
        for (int32_t f = lane; f < total; f += kWave) {
            int q = 0;
            while (f >= L.gpre[q + 1]) q++;
            const int32_t e = L.gbase[q] + (f - L.gpre[q]);
            atomicAdd((unsigned long long *)&L.conn[q][label_in(a, L, a.g.adjncy[e])], (unsigned long long)ew(a.g, e));
        }
        wave_sync();
        for (int q = 0; q < ng; q++) {
            const int32_t sl = L.gslot[q];
            long long gn;
            int32_t t;
            select_gain(a, L.conn[q], L.Bp, L.plab[sl], vw(a.g, L.qv[sl]), gn, t);
            if (lane == 0) {
                if (t >= 0) {
                    L.key[sl] = gn;
                    L.inh[sl] = 1;
                } else if (L.flag[sl] == 1) {
                    L.inh[sl] = 0;
                }
                L.flag[sl] = 0;
            }
            wave_sync();
        }
    }
}

__global__ __launch_bounds__(kWave * kSW) void k_search(SearchArgs a) {
    __shared__ WaveLds lds[kSW];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int32_t j = blockIdx.x * kSW + w;
    const int32_t ns = min(a.c->clash, a.c->nsel);
    if (j >= ns) return;  // per wavefront
    WaveLds &L = lds[w];
    for (int i = lane; i < kHT; i += kWave) L.hk[i] = -1;
    for (int b = lane; b < a.k; b += kWave) {
        for (int q = 0; q < kGG; q++) L.conn[q][b] = 0;
        L.Bp[b] = a.B[b];
    }
    L.inh[lane] = 0;
    L.flag[lane] = 0;
    wave_sync();
    const int32_t s = a.sel[j];
    // the seed, then its neighbours in adjacency order
    int32_t queued = scan_list(a, L, nullptr, 1, s, 0);
    queued = scan_list(a, L, a.g.adjncy + a.g.xadj[s], a.g.xadj[s + 1] - a.g.xadj[s], s, queued);
    eval_flags(a, L, queued);
    int32_t nlog = 0, bestlen = 0, idle = 0;
    long long cum = 0, best = 0;
    for (;;) {
        // the queued vertex of largest gain, ties -> lower id
        const bool in = lane < queued && L.inh[lane];
        long long kk = in ? L.key[lane] : LLONG_MIN;
        int32_t vv = in ? L.qv[lane] : INT_MAX;
        int32_t ss = in ? lane : -1;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const long long ok = __shfl_xor(kk, d, kWave);
            const int32_t ov = __shfl_xor(vv, d, kWave);
            const int32_t os = __shfl_xor(ss, d, kWave);
            if (ok > kk || (ok == kk && ov < vv)) {
                kk = ok;
                vv = ov;
                ss = os;
            }
        }
        if (ss < 0) break;  // queue empty
        long long gn;
        int32_t t;
        wave_gain(a, L, ss, gn, t);
        if (t < 0) {
            if (lane == 0) L.inh[ss] = 0;
            wave_sync();
            continue;
        }
        if (gn != kk) {
            if (lane == 0) L.key[ss] = gn;
            wave_sync();
            continue;
        }
        const int32_t mv = L.qv[ss];
        const int32_t from = L.plab[ss];
        const long long cw = vw(a.g, mv);
        if (lane == 0) {
            L.inh[ss] = 0;
            L.lv[nlog] = mv;
            L.lf[nlog] = from;
            L.lt[nlog] = t;
            L.Bp[from] -= cw;
            L.Bp[t] += cw;
            L.plab[ss] = t;
        }
        wave_sync();
        nlog++;
        cum += gn;
        if (cum > best) {
            best = cum;
            bestlen = nlog;
            idle = 0;
        } else if (++idle >= a.max_idle) {
            break;
        }
        queued = scan_list(a, L, a.g.adjncy + a.g.xadj[mv], a.g.xadj[mv + 1] - a.g.xadj[mv], mv, queued);
        eval_flags(a, L, queued);
    }
    const int64_t o = (int64_t)j * kMlsMaxQueue;
    if (lane < bestlen) {
        a.mv_v[o + lane] = L.lv[lane];
        a.mv_f[o + lane] = L.lf[lane];
        a.mv_t[o + lane] = L.lt[lane];
    }
    if (lane < queued) a.mk_v[o + lane] = L.qv[lane];
    if (lane == 0) {
        a.mv_n[j] = bestlen;
        a.mk_n[j] = queued;
    }
}

struct ApplyArgs {
    MG g;
    int32_t k;
    int64_t lmax;
    int32_t *part;
    int64_t *B;
    int32_t *marked, *marklist, *next;
    Ctl *c;
    const int32_t *selpos;
    const int32_t *mv_v, *mv_f, *mv_t, *mv_n, *mk_v, *mk_n;
};

__device__ __forceinline__ int32_t ld_part(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ApplyMoves: the batch's kept prefixes in seed order, every gain recomputed
// on the current partition; a prefix is cut at a vertex that already left its
// block or a target without room, and kept up to its best recomputed gain.
__global__ __launch_bounds__(kAB) void k_apply(ApplyArgs a) {
    __shared__ long long sB[kMlsMaxK];
    __shared__ long long red[2][kAB / kWave];
    const int32_t nsel = a.c->nsel;
    if (nsel == 0) {
        if (threadIdx.x == 0) a.c->ti = a.c->ntodo;
        return;
    }
    const int32_t ns = min(a.c->clash, nsel);
    for (int b = threadIdx.x; b < a.k; b += kAB) sB[b] = a.B[b];
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / kWave;
    long long lg = 0, kept = 0;
    int32_t nnext = a.c->nnext;
    for (int32_t j = 0; j < ns; j++) {
        const int64_t o = (int64_t)j * kMlsMaxQueue;
        const int32_t nm = a.mv_n[j];
        long long cum = 0, best = 0;
        int32_t na = 0, bestlen = 0;
        for (int32_t m = 0; m < nm; m++) {
            const int32_t v = a.mv_v[o + m], f = a.mv_f[o + m], t = a.mv_t[o + m];
            const long long cv = vw(a.g, v);
            if (ld_part(a.part + v) != f || sB[t] + cv > a.lmax) break;  // uniform
            long long ct = 0, cf = 0;
            for (int32_t e = a.g.xadj[v] + threadIdx.x; e < a.g.xadj[v + 1]; e += kAB) {
                const int32_t pu = ld_part(a.part + a.g.adjncy[e]);
                if (pu == t) ct += ew(a.g, e);
                else if (pu == f) cf += ew(a.g, e);
            }
            ct = wave_sum(ct);
            cf = wave_sum(cf);
            if (lane == 0) {
                red[0][w] = ct;
                red[1][w] = cf;
            }
            __syncthreads();
            ct = 0;
            cf = 0;
            for (int i = 0; i < kAB / kWave; i++) {
                ct += red[0][i];
                cf += red[1][i];
            }
            if (threadIdx.x == 0) {
                sB[f] -= cv;
                sB[t] += cv;
                __hip_atomic_store(a.part + v, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __threadfence();
            __syncthreads();
            na++;
            cum += ct - cf;
            if (cum > best) {
                best = cum;
                bestlen = na;
            }
        }
        for (int32_t i = na - 1; i >= bestlen; i--) {
            if (threadIdx.x == 0) {
                const int32_t v = a.mv_v[o + i];
                const long long cv = vw(a.g, v);
                sB[a.mv_t[o + i]] -= cv;
                sB[a.mv_f[o + i]] += cv;
                __hip_atomic_store(a.part + v, a.mv_f[o + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __threadfence();
        __syncthreads();
        for (int32_t i = threadIdx.x; i < bestlen; i += kAB) a.next[nnext + i] = a.mv_v[o + i];
        nnext += bestlen;
        lg += best;
        kept += bestlen;
    }
    // the batch's marks hold for the rest of the local iteration
    for (int32_t j = 0; j < ns; j++) {
        const int64_t o = (int64_t)j * kMlsMaxQueue;
        for (int32_t i = threadIdx.x; i < a.mk_n[j]; i += kAB) {
            const int32_t u = a.mk_v[o + i];
            if (atomicExch(&a.marked[u], 1) == 0) a.marklist[atomicAdd(&a.c->nmark, 1)] = u;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < a.k; b += kAB) a.B[b] = sB[b];
    if (threadIdx.x == 0) {
        Ctl *c = a.c;
        c->lgain += lg;
        c->kept += kept;
        c->searches += ns;
        c->nnext = nnext;
        c->ti = c->clash < nsel ? a.selpos[c->clash] : c->tiw;
        c->epoch++;
    }
}

__global__ void k_ctl_init(Ctl *c) {
    c->ti = c->ntodo = c->nsel = c->tiw = 0;
    c->clash = INT_MAX;
    c->epoch = 1;
    c->nnext = c->nmark = 0;
    c->lgain = c->kept = c->searches = 0;
}

uint64_t host_mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

}  // namespace

int mls_refine(const DevGraph &g, int32_t k, int64_t lmax, int32_t *part, int64_t *B, const int32_t *hash_id,
               uint64_t seed, int32_t global_iters, int32_t batch, int32_t queue, int32_t max_idle, double alpha,
               MlsOut *out, Scratch &sc) {
    ScratchScope scope(sc);
    hipStream_t s = sc.stream();
    MlsOut res;
    const int32_t n = g.n;
    if (n == 0 || global_iters <= 0) {
        if (out) *out = res;
        return GP_OK;
    }
    if (k < 1 || k > kMlsMaxK || queue < 1 || queue > kMlsMaxQueue || batch < 1 || batch > kMlsMaxBatch ||
        max_idle < 1) {
        set_error("mls: needs 1 <= k <= 256, 1 <= queue <= 64, 1 <= batch <= 65536 and max_idle >= 1");
        return GP_ERR_ARG;
    }
    const MG mg{g.xadj, g.adjncy, g.adjwgt, g.vwgt};
    int32_t *flag = nullptr, *todo = nullptr, *todo2 = nullptr, *next = nullptr, *marked = nullptr,
            *marklist = nullptr, *count = nullptr, *sel = nullptr, *selpos = nullptr;
    uint64_t *key = nullptr, *key2 = nullptr;
    unsigned long long *first = nullptr;
    int32_t *mv_v = nullptr, *mv_f = nullptr, *mv_t = nullptr, *mv_n = nullptr, *mk_v = nullptr, *mk_n = nullptr;
    Ctl *c = nullptr;
    GP_TRY(sc.alloc(&flag, n));
    GP_TRY(sc.alloc(&todo, n));
    GP_TRY(sc.alloc(&todo2, n));
    GP_TRY(sc.alloc(&next, n));
    GP_TRY(sc.alloc(&marked, n));
    GP_TRY(sc.alloc(&marklist, n));
    GP_TRY(sc.alloc(&count, 1));
    GP_TRY(sc.alloc(&key, n));
    GP_TRY(sc.alloc(&key2, n));
    GP_TRY(sc.alloc(&first, n));
    GP_TRY(sc.alloc(&sel, batch));
    GP_TRY(sc.alloc(&selpos, batch));
    const size_t slots = (size_t)batch * kMlsMaxQueue;
    GP_TRY(sc.alloc(&mv_v, slots));
    GP_TRY(sc.alloc(&mv_f, slots));
    GP_TRY(sc.alloc(&mv_t, slots));
    GP_TRY(sc.alloc(&mk_v, slots));
    GP_TRY(sc.alloc(&mv_n, batch));
    GP_TRY(sc.alloc(&mk_n, batch));
    GP_TRY(sc.alloc(&c, 1));
    GP_TRY(fill<int32_t>(marked, n, 0, s));
    GP_TRY(fill<unsigned long long>(first, n, ~0ull, s));
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, s, c);
    GP_LAUNCH_CHECK();

    SearchArgs sa{mg, k, lmax, part, B, marked, sel, c, queue, max_idle, mv_v, mv_f, mv_t, mv_n, mk_v, mk_n};
    ApplyArgs aa{mg, k, lmax, part, B, marked, marklist, next, c, selpos, mv_v, mv_f, mv_t, mv_n, mk_v, mk_n};
    const unsigned gsearch = (unsigned)((batch + kSW - 1) / kSW);
    constexpr int kBatchesPerCheck = 8;

    // the todo list in the hash order of (global iteration, local iteration)
    auto order = [&](int32_t gi, int32_t li) -> int {
        const uint64_t h = host_mix64(host_mix64(host_mix64(seed) ^ (uint64_t)(gi + 1)) ^ (uint64_t)(li + 1));
        hipLaunchKernelGGL(k_order_keys, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, todo, c, hash_id, h, key);
        GP_LAUNCH_CHECK();
        uint64_t *k1 = key, *k2 = key2;
        int32_t *v1 = todo, *v2 = todo2;
        GP_TRY((radix_sort<uint64_t, int32_t>(&k1, &v1, &k2, &v2, n, &c->ntodo, 64, sc)));
        if (v1 != todo) {  // 64 bits = 8 passes: the result is back in the first buffers
            set_error("mls: unexpected radix sort buffer");
            return GP_ERR_HIP;
        }
        return GP_OK;
    };

    Ctl hc;
    for (int32_t gi = 0; gi < global_iters; gi++) {
        hipLaunchKernelGGL(k_boundary, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, mg, part, n, flag);
        GP_LAUNCH_CHECK();
        GP_TRY(compact(FlagSet{flag}, EmitId{todo}, n, nullptr, count, sc));
        hipLaunchKernelGGL(k_begin_global, dim3(1), dim3(1), 0, s, c, count);
        GP_LAUNCH_CHECK();
        GP_TRY(order(gi, 0));
        int64_t gtotal = 0;
        for (int32_t li = 0;; li++) {
            res.local_iters++;
            hipLaunchKernelGGL(k_begin_local, dim3(1), dim3(1), 0, s, c);
            GP_LAUNCH_CHECK();
            for (;;) {
                for (int r = 0; r < kBatchesPerCheck; r++) {
                    hipLaunchKernelGGL(k_window, dim3(1), dim3(kAB), 0, s, todo, marked, batch, c, sel, selpos);
                    hipLaunchKernelGGL(k_claim, dim3(batch), dim3(256), 0, s, mg, sel, c, first);
                    hipLaunchKernelGGL(k_search, dim3(gsearch), dim3(kWave * kSW), 0, s, sa);
                    hipLaunchKernelGGL(k_apply, dim3(1), dim3(kAB), 0, s, aa);
                    GP_LAUNCH_CHECK();
                }
                GP_HIP(hipMemcpyAsync(&hc, c, sizeof(Ctl), hipMemcpyDeviceToHost, s));
                GP_HIP(hipStreamSynchronize(s));
                if (hc.ti >= hc.ntodo) break;
            }
            hipLaunchKernelGGL(k_unmark, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, marked, marklist, c);
            hipLaunchKernelGGL(k_reset_marks, dim3(1), dim3(1), 0, s, c);
            GP_LAUNCH_CHECK();
            const int64_t lgain = hc.lgain;
            res.gain += lgain;
            // another local iteration around the moved vertices while it pays
            if (lgain > 0 && (double)lgain > alpha * (double)gtotal) {
                gtotal += lgain;
                hipLaunchKernelGGL(k_next_to_todo, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, next, todo, c);
                GP_LAUNCH_CHECK();
                GP_TRY(order(gi, li + 1));
                if (hc.nnext == 0) break;
            } else {
                break;
            }
        }
    }
    GP_HIP(hipMemcpyAsync(&hc, c, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    res.searches = hc.searches;
    res.moves = hc.kept;
    if (out) *out = res;
    return GP_OK;
}

}  // namespace gp
