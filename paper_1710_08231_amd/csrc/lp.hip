// lp.hip — round-synchronous size-constrained label propagation on gfx950.
//
// One round (clustering §III-A / §IV-A, refinement §III-C use the same
// kernels; only the label domain and the capacity differ):
//   1. propose: per vertex, neighbour-label connection weights are gathered
//      into an LDS hash table (vertices binned by degree: a few lanes, a whole
//      wave, or a whole workgroup per vertex; vertices above the LDS tiers use
//      a table in global memory). Best = max connection, ties -> smallest
//      label; the capacity check W[L] + c(v) <= U is evaluated on the best
//      label first and only rescans the table when that label is full.
//   2. compact the movers in ascending vertex id (stable scan),
//   3. stable LSD radix sort of (target, vertex) by target, so each target's
//      proposers stay in ascending id,
//   4. inclusive prefix sum of c over the sorted movers; a mover is admitted
//      iff W[t] + (its prefix within the target's segment) <= U,
//   5. apply: write labels, then update W with integer atomics (exact,
//      order independent), count moves, update the device stop flag.
// No host synchronisation happens between rounds; after the stop flag is set
// every later kernel of the call returns immediately.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <string>

#include "lp.hpp"
#include "prims.hpp"

namespace gp {

namespace {

// per-group round bookkeeping: gs[q] = {moves this round, previous moves, done, rounds_run, rounds seen}
struct GroupState {
    int32_t moves, prev, done, rounds_run, seen;
    int64_t total;
};

struct LPArgs {
    const int32_t *xadj, *adjncy, *adjwgt, *vwgt;
    const int32_t *labels;
    const int64_t *W;
    int64_t U;
    int32_t dir_alternate;  // even rounds: only smaller labels; odd rounds: only larger labels
    int32_t *prop;
    const int32_t *done;
    const int32_t *round;  // device round counter (rounds replay one captured launch sequence)
    const int64_t *capv;   // optional per-label capacity (batched graphs); null: every label has U
    const uint8_t *lab8;   // dense mode (<= 256 labels): byte copy of labels for the neighbour gathers
    const uint8_t *act;    // active-set rounds: evaluations each vertex still owes (0: no proposal); null: all
    const int32_t *group;  // batched graphs: group of each vertex; null: one graph
    const GroupState *gs;  // batched graphs: per-group state
};

// An inactive vertex makes no proposal: its edge range is taken as empty.
// A group that stopped (two idle rounds) stays idle: its state is a fixed
// point of the rounds, and its labels and weights are its own, so evaluating
// its vertices again could only yield proposals refused as before.
__device__ __forceinline__ bool inactive(const LPArgs &a, int32_t v) {
    return (a.act && a.act[v] == 0) || (a.group && a.gs[a.group[v]].done);
}

// Vertices of the degree tiers: tier t is verts[ts[t] .. ts[t+1]), both on the
// device, so a recorded round can read lists rebuilt every round (active-set
// rounds keep only the vertices that owe an evaluation).
struct TierList {
    const int32_t *verts;
    const int64_t *ts;
};

__device__ __forceinline__ int64_t capof(const LPArgs &a, int32_t L) { return a.capv ? a.capv[L] : a.U; }

// 0: any direction, 1: only smaller labels, 2: only larger labels
__device__ __forceinline__ int32_t cur_dirmode(const LPArgs &a) {
    return a.dir_alternate ? (((*a.round) & 1) == 0 ? 1 : 2) : 0;
}

__device__ __forceinline__ bool dir_ok(int32_t L, int32_t own, int32_t dirmode) {
    return dirmode == 0 || (dirmode == 1 ? (L < own) : (L > own));
}

__device__ __forceinline__ int64_t vweight(const int32_t *vwgt, int32_t v) {
    return vwgt ? (int64_t)vwgt[v] : (int64_t)1;
}

template <typename AccT>
__device__ __forceinline__ void lds_add(AccT *p, AccT w);
template <>
__device__ __forceinline__ void lds_add<int32_t>(int32_t *p, int32_t w) {
    atomicAdd(p, w);
}
template <>
__device__ __forceinline__ void lds_add<int64_t>(int64_t *p, int64_t w) {
    atomicAdd((unsigned long long *)p, (unsigned long long)w);
}

__device__ __forceinline__ uint32_t hash_label(int32_t L) { return (uint32_t)L * 0x9E3779B1u; }

// Open addressing with linear probing; capacity (a power of two) > distinct keys.
template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename AccT>
__device__ __forceinline__ void tbl_insert(int32_t *key, AccT *val, uint32_t cap_mask, int log2cap,
                                           int32_t L, AccT w) {
    uint32_t h = hash_label(L) >> (32 - log2cap);
    for (;;) {
        int32_t k = key[h];
        if (k == L) break;
        if (k == -1) {
            int32_t prev = atomicCAS(&key[h], -1, L);
            if (prev == -1 || prev == L) break;
        }
        h = (h + 1) & cap_mask;
    }
    lds_add<AccT>(&val[h], w);
}

template <typename AccT>
__device__ __forceinline__ void tbl_insert_global(int32_t *key, AccT *val, uint32_t cap_mask, int log2cap,
                                                  int32_t L, AccT w) {
    uint32_t h = hash_label(L) >> (32 - log2cap);
    for (;;) {  // one L2 round trip per probe: the CAS result says empty, ours, or taken
        const int32_t prev = atomicCAS(&key[h], -1, L);
        if (prev == -1 || prev == L) break;
        h = (h + 1) & cap_mask;
    }
    lds_add<AccT>(&val[h], w);
}

// (conn, label) order: larger conn first, then smaller label.
template <typename AccT>
__device__ __forceinline__ bool better(AccT c, int32_t L, AccT bc, int32_t bl) {
    return c > bc || (c == bc && L < bl);
}

template <int GL, typename AccT>
__device__ __forceinline__ void group_best(AccT &bc, int32_t &bl) {
#pragma unroll
    for (int d = GL / 2; d > 0; d >>= 1) {
        AccT oc = __shfl_xor(bc, d, GL);
        int32_t ol = __shfl_xor(bl, d, GL);
        if (better(oc, ol, bc, bl)) {
            bc = oc;
            bl = ol;
        }
    }
}

template <int GL, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
    for (int d = GL / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, GL);
    return x;
}

template <int BLOCK, typename AccT>
__device__ __forceinline__ void block_best(AccT &bc, int32_t &bl, AccT *tc, int32_t *tl) {
    constexpr int NW = BLOCK / kWave;
    group_best<kWave, AccT>(bc, bl);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        tc[w] = bc;
        tl[w] = bl;
    }
    __syncthreads();
    bc = tc[0];
    bl = tl[0];
    for (int i = 1; i < NW; i++)
        if (better(tc[i], tl[i], bc, bl)) {
            bc = tc[i];
            bl = tl[i];
        }
    __syncthreads();
}

constexpr int kPropBlock = 256;
constexpr int kSmallLabels = 4096;  // label counts handled with per-block LDS totals
constexpr int kDenseLabels = 256;   // label counts handled with dense per-vertex tables

// GL lanes per vertex (GL <= 64), TBL table slots per vertex.
template <int GL, int TBL, typename AccT>
__global__ __launch_bounds__(kPropBlock) void k_propose_group(LPArgs a, TierList lists, int tier) {
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int GPW = kWave / GL;
    constexpr int NW = kPropBlock / kWave;
    constexpr int LOG2 = __builtin_ctz(TBL);
    __shared__ int32_t skey[NW * GPW * TBL];
    __shared__ AccT sval[NW * GPW * TBL];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int gl = lane % GL, grp = lane / GL;
    int32_t *key = skey + (w * GPW + grp) * TBL;
    AccT *val = sval + (w * GPW + grp) * TBL;
    for (int i = gl; i < TBL; i += GL) {
        key[i] = -1;
        val[i] = 0;
    }
    wave_sync();
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * NW * GPW;
    for (int64_t wb = ((int64_t)b * NW + w) * GPW; wb < count; wb += stride) {
        const int64_t idx = wb + grp;
        const bool valid = idx < count;
        const int32_t v = valid ? verts[idx] : 0;
        const int32_t beg = valid ? a.xadj[v] : 0;
        const int32_t end = (valid && !inactive(a, v)) ? a.xadj[v + 1] : beg;
        const int32_t own = valid ? a.labels[v] : -1;
        AccT oc = 0;
        const int nch = (end - beg + GL - 1) / GL;
        const int maxch = wave_max(nch);
        for (int ch = 0; ch < maxch; ch += 2) {
            const int32_t e0 = beg + ch * GL + gl, e1 = e0 + GL;
            const int32_t u0 = e0 < end ? a.adjncy[e0] : -1, u1 = e1 < end ? a.adjncy[e1] : -1;
            const AccT w0 = (e0 < end && a.adjwgt) ? (AccT)a.adjwgt[e0] : (AccT)1;
            const AccT w1 = (e1 < end && a.adjwgt) ? (AccT)a.adjwgt[e1] : (AccT)1;
            const int32_t L0 = u0 >= 0 ? a.labels[u0] : -1, L1 = u1 >= 0 ? a.labels[u1] : -1;
            if (u0 >= 0) {
                if (L0 == own) oc += w0;
                else if (dir_ok(L0, own, dmode)) tbl_insert<AccT>(key, val, TBL - 1, LOG2, L0, w0);
            }
            if (u1 >= 0) {
                if (L1 == own) oc += w1;
                else if (dir_ok(L1, own, dmode)) tbl_insert<AccT>(key, val, TBL - 1, LOG2, L1, w1);
            }
        }
        wave_sync();
        oc = group_sum<GL>(oc);
        AccT bc = 0;
        int32_t bl = INT_MAX;
        for (int i = gl; i < TBL; i += GL) {
            const int32_t L = key[i];
            if (L >= 0 && better(val[i], L, bc, bl)) {
                bc = val[i];
                bl = L;
            }
        }
        group_best<GL, AccT>(bc, bl);
        const int64_t cv = valid ? vweight(a.vwgt, v) : 0;
        int32_t target = -1;
        bool need2 = false;
        if (valid && bl != INT_MAX && bc > oc) {
            if (a.W[bl] + cv <= capof(a, bl)) target = bl;
            else need2 = true;
        }
        if (__ballot(need2)) {
            AccT bc2 = 0;
            int32_t bl2 = INT_MAX;
            if (need2) {
                for (int i = gl; i < TBL; i += GL) {
                    const int32_t L = key[i];
                    if (L >= 0 && better(val[i], L, bc2, bl2) && a.W[L] + cv <= capof(a, L)) {
                        bc2 = val[i];
                        bl2 = L;
                    }
                }
            }
            group_best<GL, AccT>(bc2, bl2);
            if (need2 && bl2 != INT_MAX && bc2 > oc) target = bl2;
        }
        if (valid && gl == 0) a.prop[v] = target;
        wave_sync();
        for (int i = gl; i < TBL; i += GL) {
            key[i] = -1;
            val[i] = 0;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------- packed tables (32-bit sums)
//
// With 32-bit connection sums a table slot is one 64-bit LDS word, label in
// the high half and connection in the low half (an empty slot holds label
// 0xFFFFFFFF), so an insert is one CAS (new label) or one 64-bit add (known
// label) that returns the label's running sum. The largest connection (ties:
// smallest label) is then known without scanning the table: every lane keeps
// the maximum of the sums its own adds returned, packed as (sum << 32 | ~label);
// the last add to a label returns its final sum, so the maximum over the lanes
// is the maximum over the labels. Each lane remembers the slots it touched and
// clears them afterwards. The table is scanned only when the best label has no
// room under its bound (then for the best label with room), exactly as before.
constexpr unsigned long long kSlotEmpty = 0xFFFFFFFF00000000ull;

__device__ __forceinline__ unsigned long long pack_best(uint32_t c, int32_t L) {
    return ((unsigned long long)c << 32) | (uint32_t)(~(uint32_t)L);
}

// Adds w to label L's slot (inserting it); returns the slot, *sum the label's sum after the add.
__device__ __forceinline__ uint32_t slot_add(unsigned long long *tbl, uint32_t mask, int lg, int32_t L, uint32_t w,
                                             uint32_t *sum) {
    uint32_t h = hash_label(L) >> (32 - lg);
    for (;;) {
        unsigned long long cur = tbl[h];
        if (cur == kSlotEmpty) {
            cur = atomicCAS(&tbl[h], kSlotEmpty, ((unsigned long long)(uint32_t)L << 32) | w);
            if (cur == kSlotEmpty) {
                *sum = w;
                return h;
            }
        }
        if ((uint32_t)(cur >> 32) == (uint32_t)L) {
            *sum = (uint32_t)atomicAdd(&tbl[h], (unsigned long long)w) + w;
            return h;
        }
        h = (h + 1) & mask;
    }
}

// The best label with room for a vertex of weight cv among the table slots
// first, first + step, ... below cap (ties: lower label). A slot is a
// candidate when it beats the best found so far; the weights of up to four
// candidates are requested together, so a lane waits on memory once per four
// slots, not once per candidate. The result is the maximum over the eligible
// labels and does not depend on the order of the slots.
__device__ __forceinline__ void best_with_room(const LPArgs &a, const unsigned long long *tbl, uint32_t first,
                                               uint32_t step, uint32_t cap, int64_t cv, int32_t &bc2,
                                               int32_t &bl2) {
    for (uint32_t i0 = first; i0 < cap; i0 += 4 * step) {
        int32_t L[4], c[4];
        int64_t wl[4], cl[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t i = i0 + q * step;
            L[q] = -1;
            c[q] = 0;
            if (i < cap) {
                const unsigned long long sl = tbl[i];
                if (sl != kSlotEmpty) {
                    L[q] = (int32_t)(sl >> 32);
                    c[q] = (int32_t)(uint32_t)sl;
                    if (!better(c[q], L[q], bc2, bl2)) L[q] = -1;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            wl[q] = L[q] >= 0 ? a.W[L[q]] : 0;
            cl[q] = L[q] >= 0 ? capof(a, L[q]) : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (L[q] >= 0 && wl[q] + cv <= cl[q] && better(c[q], L[q], bc2, bl2)) {
                bc2 = c[q];
                bl2 = L[q];
            }
    }
}

template <int GL>
__device__ __forceinline__ unsigned long long group_max_u64(unsigned long long x) {
#pragma unroll
    for (int d = GL / 2; d > 0; d >>= 1) {
        const unsigned long long y = __shfl_xor(x, d, GL);
        x = y > x ? y : x;
    }
    return x;
}

// GL lanes per vertex, TBL packed slots per vertex (degrees up to TBL / 2).
template <int GL, int TBL>
__global__ __launch_bounds__(kPropBlock) void k_pgroup(LPArgs a, TierList lists, int tier) {
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int GPW = kWave / GL;
    constexpr int NW = kPropBlock / kWave;
    constexpr int LOG2 = __builtin_ctz(TBL);
    constexpr int MAXE = 2 * ((TBL / 2 + 2 * GL - 1) / (2 * GL));  // entries per lane and vertex
    __shared__ unsigned long long stbl[NW * GPW * TBL];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int gl = lane % GL, grp = lane / GL;
    unsigned long long *tbl = stbl + (w * GPW + grp) * TBL;
    for (int i = gl; i < TBL; i += GL) tbl[i] = kSlotEmpty;
    wave_sync();
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * NW * GPW;
    for (int64_t wb = ((int64_t)b * NW + w) * GPW; wb < count; wb += stride) {
        const int64_t idx = wb + grp;
        const bool valid = idx < count;
        const int32_t v = valid ? verts[idx] : 0;
        const int32_t beg = valid ? a.xadj[v] : 0;
        const int32_t end = (valid && !inactive(a, v)) ? a.xadj[v + 1] : beg;
        const int32_t own = valid ? a.labels[v] : -1;
        int32_t oc = 0;
        unsigned long long mybest = 0;
        uint32_t touched[MAXE];  // fixed positions (registers): entry it*2 + j, ~0u when none
        const int nch = (end - beg + GL - 1) / GL;
        const int maxch = wave_max(nch);
#pragma unroll
        for (int it = 0; it < MAXE / 2; it++) {
            touched[2 * it] = ~0u;
            touched[2 * it + 1] = ~0u;
            if (2 * it >= maxch) continue;
            const int32_t e0 = beg + 2 * it * GL + gl, e1 = e0 + GL;
            const int32_t u0 = e0 < end ? a.adjncy[e0] : -1, u1 = e1 < end ? a.adjncy[e1] : -1;
            const int32_t w0 = (e0 < end && a.adjwgt) ? a.adjwgt[e0] : 1;
            const int32_t w1 = (e1 < end && a.adjwgt) ? a.adjwgt[e1] : 1;
            const int32_t L0 = u0 >= 0 ? a.labels[u0] : -1, L1 = u1 >= 0 ? a.labels[u1] : -1;
            uint32_t sum;
            if (u0 >= 0) {
                if (L0 == own) oc += w0;
                else if (dir_ok(L0, own, dmode)) {
                    touched[2 * it] = slot_add(tbl, TBL - 1, LOG2, L0, (uint32_t)w0, &sum);
                    const unsigned long long pb = pack_best(sum, L0);
                    mybest = pb > mybest ? pb : mybest;
                }
            }
            if (u1 >= 0) {
                if (L1 == own) oc += w1;
                else if (dir_ok(L1, own, dmode)) {
                    touched[2 * it + 1] = slot_add(tbl, TBL - 1, LOG2, L1, (uint32_t)w1, &sum);
                    const unsigned long long pb = pack_best(sum, L1);
                    mybest = pb > mybest ? pb : mybest;
                }
            }
        }
        wave_sync();
        oc = group_sum<GL>(oc);
        mybest = group_max_u64<GL>(mybest);
        const int32_t bc = (int32_t)(mybest >> 32);
        const int32_t bl = mybest ? (int32_t)~(uint32_t)mybest : INT_MAX;
        const int64_t cv = valid ? vweight(a.vwgt, v) : 0;
        int32_t target = -1;
        bool need2 = false;
        if (valid && bl != INT_MAX && bc > oc) {
            if (a.W[bl] + cv <= capof(a, bl)) target = bl;
            else need2 = true;
        }
        if (__ballot(need2)) {
            int32_t bc2 = 0, bl2 = INT_MAX;
            if (need2) {
                for (int i = gl; i < TBL; i += GL) {
                    const unsigned long long sl = tbl[i];
                    if (sl == kSlotEmpty) continue;
                    const int32_t L = (int32_t)(sl >> 32), c = (int32_t)(uint32_t)sl;
                    if (better(c, L, bc2, bl2) && a.W[L] + cv <= capof(a, L)) {
                        bc2 = c;
                        bl2 = L;
                    }
                }
            }
            group_best<GL, int32_t>(bc2, bl2);
            if (need2 && bl2 != INT_MAX && bc2 > oc) target = bl2;
        }
        if (valid && gl == 0) a.prop[v] = target;
        wave_sync();
#pragma unroll
        for (int i = 0; i < MAXE; i++)
            if (touched[i] != ~0u) tbl[touched[i]] = kSlotEmpty;
        wave_sync();
    }
}

// Tiers of at most E neighbours (4 or 8, E <= GL), 32-bit sums: one entry per
// lane, so a label's connection is summed over the group's first E lanes by
// shuffles and no table is written, read or cleared. Each lane offers its own
// label (lanes of one label offer the same sum), and the rule is that of
// k_pgroup: the strongest label other than its own, if it beats the own
// label's sum and has room, else the strongest with room. The next vertex's
// row and entry are loaded while the current one is selected. (With 16 lanes
// the shuffles cost more than the table: the tier of up to 16 neighbours keeps
// k_pgroup.)
template <int GL, int E>
__global__ __launch_bounds__(kPropBlock) void k_plane(LPArgs a, TierList lists, int tier) {
    static_assert(E <= GL, "one entry per lane");
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int GPW = kWave / GL;
    constexpr int NW = kPropBlock / kWave;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int gl = lane % GL, grp = lane / GL;
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * NW * GPW;
    int64_t wb = ((int64_t)b * NW + w) * GPW;
    bool valid = wb + grp < count;
    int32_t v = valid ? verts[wb + grp] : 0;
    int32_t beg = valid ? a.xadj[v] : 0;
    int32_t end = (valid && !inactive(a, v)) ? a.xadj[v + 1] : beg;
    int32_t own = valid ? a.labels[v] : -1;
    int32_t u = beg + gl < end ? a.adjncy[beg + gl] : -1;
    int32_t wt = (u >= 0 && a.adjwgt) ? a.adjwgt[beg + gl] : 1;
    int32_t L = u >= 0 ? a.labels[u] : -1;
    for (; wb < count; wb += stride) {
        // the next vertex's row, label and entry
        const int64_t nwb = wb + stride;
        const bool nvalid = nwb + grp < count;
        const int32_t nv = nvalid ? verts[nwb + grp] : 0;
        const int32_t nbeg = nvalid ? a.xadj[nv] : 0;
        const int32_t nend = (nvalid && !inactive(a, nv)) ? a.xadj[nv + 1] : nbeg;
        const int32_t nown = nvalid ? a.labels[nv] : -1;
        const int32_t nu = nbeg + gl < nend ? a.adjncy[nbeg + gl] : -1;
        const int32_t nwt = (nu >= 0 && a.adjwgt) ? a.adjwgt[nbeg + gl] : 1;
        int32_t c = 0;
#pragma unroll
        for (int d = 0; d < E; d++) {
            const int32_t Ld = __shfl(L, d, GL);
            const int32_t wd = __shfl(wt, d, GL);
            if (Ld == L) c += wd;
        }
        const int32_t oc = group_sum<GL>((L >= 0 && L == own) ? wt : 0);
        const bool cand = L >= 0 && L != own && dir_ok(L, own, dmode);
        const unsigned long long best = group_max_u64<GL>(cand ? pack_best((uint32_t)c, L) : 0ull);
        const int32_t bc = (int32_t)(best >> 32);
        const int32_t bl = best ? (int32_t)~(uint32_t)best : INT_MAX;
        const int64_t cv = valid ? vweight(a.vwgt, v) : 0;
        int32_t target = -1;
        bool need2 = false;
        if (valid && bl != INT_MAX && bc > oc) {
            if (a.W[bl] + cv <= capof(a, bl)) target = bl;
            else need2 = true;
        }
        if (__ballot(need2)) {
            int32_t bc2 = 0, bl2 = INT_MAX;
            if (need2 && cand && a.W[L] + cv <= capof(a, L)) {
                bc2 = c;
                bl2 = L;
            }
            group_best<GL, int32_t>(bc2, bl2);
            if (need2 && bl2 != INT_MAX && bc2 > oc) target = bl2;
        }
        if (valid && gl == 0) a.prop[v] = target;
        valid = nvalid;
        v = nv;
        own = nown;
        u = nu;
        wt = nwt;
        L = nu >= 0 ? a.labels[nu] : -1;
    }
}

// One workgroup per vertex, BLOCK threads, packed table of the next power of
// two >= 2*deg slots (at most TBL). The loads are pipelined over the
// workgroup's vertices: the next vertex's neighbour ids and weights are
// requested before the current vertex's selection, its neighbour labels
// during it, so a vertex's memory latency overlaps the previous vertex's
// reductions and barriers.
template <int BLOCK, int TBL>
__global__ __launch_bounds__(BLOCK) void k_pblock(LPArgs a, TierList lists, int tier) {
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int NW = BLOCK / kWave;
    constexpr int MAXE = 4 * ((TBL / 2 + 4 * BLOCK - 1) / (4 * BLOCK));  // entries per thread
    __shared__ unsigned long long tbl[TBL];
    __shared__ unsigned long long wbest[NW];
    __shared__ int32_t tc[NW + 1];
    __shared__ int32_t tl[NW + 1];
    for (int i = threadIdx.x; i < TBL; i += BLOCK) tbl[i] = kSlotEmpty;
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int64_t idx = xcd_block(blockIdx.x, gridDim.x);
    int32_t v = idx < count ? verts[idx] : 0;
    int32_t beg = idx < count ? a.xadj[v] : 0, end = idx < count ? a.xadj[v + 1] : 0;
    int32_t own = idx < count ? a.labels[v] : -1;
    if (idx < count && inactive(a, v)) end = beg;
    // entry it of this thread is beg + threadIdx.x + it * BLOCK
    int32_t L[MAXE], wv[MAXE];
    {
        int32_t u[MAXE];
#pragma unroll
        for (int it = 0; it < MAXE; it++) {
            const int32_t e = beg + (int32_t)threadIdx.x + it * BLOCK;
            u[it] = e < end ? a.adjncy[e] : -1;
            wv[it] = (e < end && a.adjwgt) ? a.adjwgt[e] : 1;
        }
#pragma unroll
        for (int it = 0; it < MAXE; it++) L[it] = u[it] >= 0 ? a.labels[u[it]] : -2;
    }
    for (; idx < count; idx += gridDim.x) {
        const int64_t nidx = idx + gridDim.x;
        const int32_t nv = nidx < count ? verts[nidx] : 0;
        int lg = 6;
        while ((1 << lg) < 2 * (end - beg) && (1 << lg) < TBL) lg++;
        const uint32_t cap = 1u << lg;
        int32_t oc = 0;
        unsigned long long mybest = 0;
        uint32_t touched[MAXE];  // fixed positions (registers), ~0u when none
#pragma unroll
        for (int it = 0; it < MAXE; it++) {
            touched[it] = ~0u;
            if (L[it] == -2) continue;  // no entry
            if (L[it] == own) oc += wv[it];
            else if (dir_ok(L[it], own, dmode)) {
                uint32_t sum;
                touched[it] = slot_add(tbl, cap - 1, lg, L[it], (uint32_t)wv[it], &sum);
                const unsigned long long pb = pack_best(sum, L[it]);
                mybest = pb > mybest ? pb : mybest;
            }
        }
        // the next vertex: row, label, then its neighbour ids and weights
        const int32_t nbeg = nidx < count ? a.xadj[nv] : 0;
        int32_t nend = nidx < count ? a.xadj[nv + 1] : 0;
        const int32_t nown = nidx < count ? a.labels[nv] : -1;
        if (nidx < count && inactive(a, nv)) nend = nbeg;
        int32_t nu[MAXE];
#pragma unroll
        for (int it = 0; it < MAXE; it++) {
            const int32_t e = nbeg + (int32_t)threadIdx.x + it * BLOCK;
            nu[it] = e < nend ? a.adjncy[e] : -1;
            wv[it] = (e < nend && a.adjwgt) ? a.adjwgt[e] : 1;  // this vertex's weights are no longer needed
        }
        mybest = group_max_u64<kWave>(mybest);
        if (lane == 0) wbest[w] = mybest;
        oc = block_sum<BLOCK>(oc, tc);  // its barriers also publish wbest and the table
        // the next vertex's neighbour labels are in flight during the selection
#pragma unroll
        for (int it = 0; it < MAXE; it++) L[it] = nu[it] >= 0 ? a.labels[nu[it]] : -2;
        unsigned long long best = wbest[0];
        for (int i = 1; i < NW; i++) best = wbest[i] > best ? wbest[i] : best;
        const int32_t bc = (int32_t)(best >> 32);
        const int32_t bl = best ? (int32_t)~(uint32_t)best : INT_MAX;
        const int64_t cv = vweight(a.vwgt, v);
        int32_t target = -1;
        if (bl != INT_MAX && bc > oc) {
            if (a.W[bl] + cv <= capof(a, bl)) {
                target = bl;
            } else {
                int32_t bc2 = 0, bl2 = INT_MAX;
                best_with_room(a, tbl, threadIdx.x, BLOCK, cap, cv, bc2, bl2);
                block_best<BLOCK, int32_t>(bc2, bl2, tc, tl);
                if (bl2 != INT_MAX && bc2 > oc) target = bl2;
            }
        }
        if (threadIdx.x == 0) a.prop[v] = target;
        __syncthreads();  // every lane has read the table and wbest
#pragma unroll
        for (int i = 0; i < MAXE; i++)
            if (touched[i] != ~0u) tbl[touched[i]] = kSlotEmpty;
        __syncthreads();
        v = nv;
        beg = nbeg;
        end = nend;
        own = nown;
    }
}

// One workgroup per vertex, table in LDS sized to the vertex: next power of
// two >= 2*deg (at most TBL), so scanning and clearing cost O(deg).
template <int BLOCK, int TBL, typename AccT>
__global__ __launch_bounds__(BLOCK) void k_propose_block(LPArgs a, TierList lists, int tier) {
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int NW = BLOCK / kWave;
    constexpr int U4 = 4;
    __shared__ int32_t key[TBL];
    __shared__ AccT val[TBL];
    __shared__ AccT tc[NW + 1];
    __shared__ int32_t tl[NW + 1];
    for (int i = threadIdx.x; i < TBL; i += BLOCK) {
        key[i] = -1;
        val[i] = 0;
    }
    __syncthreads();
    // the next vertex's id is loaded with the current vertex's edges, and its
    // row range and label during the current selection, so each vertex
    // starts with its edge loads
    int64_t idx = xcd_block(blockIdx.x, gridDim.x);
    int32_t v = idx < count ? verts[idx] : 0;
    int32_t beg = idx < count ? a.xadj[v] : 0, end = idx < count ? a.xadj[v + 1] : 0;
    int32_t own = idx < count ? a.labels[v] : -1;
    for (; idx < count; idx += gridDim.x) {
        const int64_t nidx = idx + gridDim.x;
        const int32_t nv = nidx < count ? verts[nidx] : 0;
        if (inactive(a, v)) end = beg;
        int lg = 6;
        while ((1 << lg) < 2 * (end - beg) && (1 << lg) < TBL) lg++;
        const uint32_t cap = 1u << lg;
        AccT oc = 0;
        for (int32_t e0 = beg + threadIdx.x; e0 < end; e0 += U4 * BLOCK) {
            int32_t u[U4], L[U4];
            AccT wv[U4];
#pragma unroll
            for (int j = 0; j < U4; j++) {
                const int32_t e = e0 + j * BLOCK;
                u[j] = e < end ? a.adjncy[e] : -1;
                wv[j] = (e < end && a.adjwgt) ? (AccT)a.adjwgt[e] : (AccT)1;
            }
#pragma unroll
            for (int j = 0; j < U4; j++) L[j] = u[j] >= 0 ? a.labels[u[j]] : -1;
#pragma unroll
            for (int j = 0; j < U4; j++) {
                if (u[j] < 0) continue;
                if (L[j] == own) oc += wv[j];
                else if (dir_ok(L[j], own, dmode)) tbl_insert<AccT>(key, val, cap - 1, lg, L[j], wv[j]);
            }
        }
        __syncthreads();
        const int32_t nbeg = nidx < count ? a.xadj[nv] : 0, nend = nidx < count ? a.xadj[nv + 1] : 0;
        const int32_t nown = nidx < count ? a.labels[nv] : -1;
        oc = block_sum<BLOCK>(oc, tc);
        AccT bc = 0;
        int32_t bl = INT_MAX;
        for (uint32_t i = threadIdx.x; i < cap; i += BLOCK) {
            const int32_t L = key[i];
            if (L >= 0 && better(val[i], L, bc, bl)) {
                bc = val[i];
                bl = L;
            }
        }
        block_best<BLOCK, AccT>(bc, bl, tc, tl);
        const int64_t cv = vweight(a.vwgt, v);
        int32_t target = -1;
        if (bl != INT_MAX && bc > oc) {
            if (a.W[bl] + cv <= capof(a, bl)) {
                target = bl;
            } else {
                AccT bc2 = 0;
                int32_t bl2 = INT_MAX;
                for (uint32_t i = threadIdx.x; i < cap; i += BLOCK) {
                    const int32_t L = key[i];
                    if (L >= 0 && better(val[i], L, bc2, bl2) && a.W[L] + cv <= capof(a, L)) {
                        bc2 = val[i];
                        bl2 = L;
                    }
                }
                block_best<BLOCK, AccT>(bc2, bl2, tc, tl);
                if (bl2 != INT_MAX && bc2 > oc) target = bl2;
            }
        }
        if (threadIdx.x == 0) a.prop[v] = target;
        for (uint32_t i = threadIdx.x; i < cap; i += BLOCK) {
            key[i] = -1;
            val[i] = 0;
        }
        __syncthreads();
        v = nv;
        beg = nbeg;
        end = nend;
        own = nown;
    }
}

// Hubs: one workgroup per vertex, table of hcap[i] (power of two) slots in
// global memory at hoff[i]; tables start empty and are emptied again.
template <int BLOCK, typename AccT>
__global__ __launch_bounds__(BLOCK) void k_propose_hub(LPArgs a, const int32_t *__restrict__ verts,
                                                       int32_t count, const int64_t *hoff,
                                                       const int32_t *hlog, int32_t *gkey, AccT *gval) {
    if (*a.done) return;
    const int32_t dmode = cur_dirmode(a);
    constexpr int NW = BLOCK / kWave;
    __shared__ AccT tc[NW + 1];
    __shared__ int32_t tl[NW + 1];
    for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int32_t v = verts[idx];
        if (inactive(a, v)) {  // uniform per workgroup: its table stays empty
            if (threadIdx.x == 0) a.prop[v] = -1;
            continue;
        }
        const int32_t beg = a.xadj[v], end = a.xadj[v + 1];
        const int32_t own = a.labels[v];
        const int lg = hlog[idx];
        const uint32_t cap = 1u << lg;
        int32_t *key = gkey + hoff[idx];
        AccT *val = gval + hoff[idx];
        AccT oc = 0;
        for (int32_t e = beg + threadIdx.x; e < end; e += BLOCK) {
            const int32_t u = a.adjncy[e];
            const AccT wgt = a.adjwgt ? (AccT)a.adjwgt[e] : (AccT)1;
            const int32_t L = a.labels[u];
            if (L == own) oc += wgt;
            else if (dir_ok(L, own, dmode)) tbl_insert_global<AccT>(key, val, cap - 1, lg, L, wgt);
        }
        __threadfence_block();
        __syncthreads();
        oc = block_sum<BLOCK>(oc, tc);
        AccT bc = 0;
        int32_t bl = INT_MAX;
        for (uint32_t i = threadIdx.x; i < cap; i += BLOCK) {
            const int32_t L = ld_agent(&key[i]);
            const AccT c = L >= 0 ? ld_agent(&val[i]) : AccT(0);
            if (L >= 0 && better(c, L, bc, bl)) {
                bc = c;
                bl = L;
            }
        }
        block_best<BLOCK, AccT>(bc, bl, tc, tl);
        const int64_t cv = vweight(a.vwgt, v);
        int32_t target = -1;
        if (bl != INT_MAX && bc > oc) {
            if (a.W[bl] + cv <= capof(a, bl)) {
                target = bl;
            } else {
                AccT bc2 = 0;
                int32_t bl2 = INT_MAX;
                for (uint32_t i = threadIdx.x; i < cap; i += BLOCK) {
                    const int32_t L = ld_agent(&key[i]);
                    const AccT c = L >= 0 ? ld_agent(&val[i]) : AccT(0);
                    if (L >= 0 && better(c, L, bc2, bl2) && a.W[L] + cv <= capof(a, L)) {
                        bc2 = c;
                        bl2 = L;
                    }
                }
                block_best<BLOCK, AccT>(bc2, bl2, tc, tl);
                if (bl2 != INT_MAX && bc2 > oc) target = bl2;
            }
        }
        if (threadIdx.x == 0) a.prop[v] = target;
        for (uint32_t i = threadIdx.x; i < cap; i += BLOCK) {
            key[i] = -1;
            val[i] = 0;
        }
        __threadfence_block();
        __syncthreads();
    }
}

// ---------------------------------------------------------------- hubs split over workgroups

// A hub's edges are cut into chunks of kHubChunk entries. Each chunk's
// workgroup sums its (label, weight) pairs in an LDS table and deals the
// distinct labels into the hub's buckets (a hash of the label picks one),
// writing each bucket's pairs as one contiguous run of that bucket's region.
// One workgroup per bucket then sums the bucket's pairs in LDS and offers the
// best label with room, packed into a 64-bit key merged with atomicMax: high
// word conn, low word INT_MAX - label, so the maximum is the largest
// connection with the smallest label. Used for 32-bit connection sums (the
// packed key needs conn < 2^31). Nothing is hashed into global memory unless a
// bucket's region overflows: its pairs then go to the hub's overflow table,
// which a third kernel scans (and empties) only for such hubs.
constexpr int kHubChunk = 4096;
constexpr int kHubSlice = 4096;
constexpr int kHubPer = 2048;       // buckets per hub: degree / kHubPer, rounded up
constexpr int kHubMaxBuck = 2048;   // at most (the insert kernel's LDS histogram)
constexpr int kBucketCap = 4096;    // pairs a bucket region holds
constexpr int kRedLds = 2 * kBucketCap;
constexpr int kRedBlock = 512;

struct HubPlan {
    const int32_t *hubs;       // [nh] hub vertex ids
    const int64_t *toff;       // [nh] overflow table offset
    const int32_t *tlog;       // [nh] log2 overflow table capacity
    const int32_t *chunk_hub;  // [nchunks]
    const int32_t *chunk_first;  // [nh] first chunk of hub
    const int32_t *slice_hub;  // [nslices] overflow table slices
    const int32_t *slice_first;  // [nh]
    const int32_t *nbk;        // [nh] buckets of hub
    const int32_t *bk_first;   // [nh] first bucket of hub
    const int32_t *bk_hub;     // [nbuckets]
    int32_t *fill;             // [nbuckets] pairs reserved in the bucket's region this round
    int2 *pairs;               // [nbuckets * kBucketCap] (label, conn)
    int32_t *key;              // overflow tables (all -1 between rounds)
    int32_t *val;              //   (all 0 between rounds)
    int32_t *ovf;              // [nh] a pair of the hub went to its overflow table
    unsigned long long *own;   // [nh] connection to the hub's own label
    unsigned long long *best;  // [nh] best packed (conn, label) with room
};

__device__ __forceinline__ unsigned long long pack_best(int32_t c, int32_t L) {
    return ((unsigned long long)(uint32_t)c << 32) | (unsigned long long)(uint32_t)(INT_MAX - L);
}

// Bucket of a label: MurmurHash3's 32-bit finaliser (fmix32), scaled to nb by a
// multiply-high. Independent of the top bits of hash_label that place the
// label in the LDS tables, so a bucket's labels still spread over its table.
__device__ __forceinline__ uint32_t bucket_of(int32_t L, uint32_t nb) {
    uint32_t x = (uint32_t)L;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return (uint32_t)(((uint64_t)x * nb) >> 32);
}

// One workgroup per chunk of a hub's edges; its LDS table (at most kHubLds
// slots) is sized to the chunk, so it is at most half full.
constexpr int kHubLds = 2 * kHubChunk;
constexpr int kHubLdsLog = 13;
static_assert((1 << kHubLdsLog) == kHubLds, "LDS table size");
constexpr int kHubBlock = 1024;

__global__ __launch_bounds__(kHubBlock) void k_hub_insert(LPArgs a, HubPlan hp) {
    if (*a.done) return;
    const int32_t dmode = cur_dirmode(a);
    __shared__ int32_t skey[kHubLds];
    __shared__ int32_t sval[kHubLds];
    __shared__ int32_t scur[kHubMaxBuck];
    __shared__ int32_t tmp[kHubBlock / kWave + 1];
    const int32_t h = hp.chunk_hub[blockIdx.x];
    const int32_t v = hp.hubs[h];
    if (inactive(a, v)) return;  // uniform: nothing goes into the hub's buckets
    const int32_t nb = hp.nbk[h];
    const int32_t beg = a.xadj[v] + (blockIdx.x - hp.chunk_first[h]) * kHubChunk;
    const int32_t end = min(a.xadj[v + 1], beg + kHubChunk);
    int tlg = 6;  // table sized to the chunk: next power of two >= 2 * entries
    while ((1 << tlg) < 2 * (end - beg)) tlg++;
    const int tcap = 1 << tlg;
    for (int i = threadIdx.x; i < tcap; i += kHubBlock) {
        skey[i] = -1;
        sval[i] = 0;
    }
    for (int i = threadIdx.x; i < nb; i += kHubBlock) scur[i] = 0;
    __syncthreads();
    const int32_t own = a.labels[v];
    int32_t oc = 0;
    for (int32_t e = beg + threadIdx.x; e < end; e += kHubBlock) {
        const int32_t u = a.adjncy[e];
        const int32_t wv = a.adjwgt ? a.adjwgt[e] : 1;
        const int32_t L = a.labels[u];
        if (L == own) oc += wv;
        else if (dir_ok(L, own, dmode)) tbl_insert<int32_t>(skey, sval, tcap - 1, tlg, L, wv);
    }
    __syncthreads();
    // pairs per bucket, then one reservation per non-empty bucket in its region
    for (int i = threadIdx.x; i < tcap; i += kHubBlock) {
        const int32_t L = skey[i];
        if (L >= 0) atomicAdd(&scur[bucket_of(L, (uint32_t)nb)], 1);
    }
    __syncthreads();
    const int32_t gb0 = hp.bk_first[h];
    for (int b = threadIdx.x; b < nb; b += kHubBlock) {
        const int32_t c = scur[b];
        if (c) scur[b] = atomicAdd(&hp.fill[gb0 + b], c);
    }
    __syncthreads();
    const int lg = hp.tlog[h];
    int32_t *key = hp.key + hp.toff[h];
    int32_t *val = hp.val + hp.toff[h];
    for (int i = threadIdx.x; i < tcap; i += kHubBlock) {
        const int32_t L = skey[i];
        if (L < 0) continue;
        const uint32_t b = bucket_of(L, (uint32_t)nb);
        const int32_t pos = atomicAdd(&scur[b], 1);
        if (pos < kBucketCap) {
            hp.pairs[(int64_t)(gb0 + (int32_t)b) * kBucketCap + pos] = make_int2(L, sval[i]);
        } else {  // region full: this pair goes to the hub's overflow table
            tbl_insert_global<int32_t>(key, val, (1u << lg) - 1, lg, L, sval[i]);
            hp.ovf[h] = 1;
        }
    }
    oc = block_sum<kHubBlock>(oc, tmp);
    if (threadIdx.x == 0 && oc) atomicAdd(&hp.own[h], (unsigned long long)oc);
}

// One workgroup per bucket: sum its pairs in an LDS table sized to them and
// offer the best label with room (W at the round start, as every proposal
// kernel tests it). An overflowed bucket instead moves the pairs of its region
// to the hub's overflow table, where the rest of them already are. Empties the
// bucket for the next round.
__global__ __launch_bounds__(kRedBlock) void k_hub_reduce(LPArgs a, HubPlan hp) {
    if (*a.done) return;
    __shared__ int32_t skey[kRedLds];
    __shared__ int32_t sval[kRedLds];
    __shared__ unsigned long long tmp[kRedBlock / kWave + 1];
    const int32_t gb = blockIdx.x;
    const int32_t f = hp.fill[gb];
    if (f == 0) return;  // uniform
    const int32_t h = hp.bk_hub[gb];
    const int2 *pr = hp.pairs + (int64_t)gb * kBucketCap;
    if (f > kBucketCap) {
        const int lg = hp.tlog[h];
        int32_t *key = hp.key + hp.toff[h];
        int32_t *val = hp.val + hp.toff[h];
        for (int i = threadIdx.x; i < kBucketCap; i += kRedBlock) {
            const int2 p = pr[i];
            tbl_insert_global<int32_t>(key, val, (1u << lg) - 1, lg, p.x, p.y);
        }
        __syncthreads();
        if (threadIdx.x == 0) hp.fill[gb] = 0;
        return;
    }
    int lg = 8;
    while ((1 << lg) < 2 * f) lg++;  // f <= kBucketCap, so lg <= log2(kRedLds)
    const int cap = 1 << lg;
    for (int i = threadIdx.x; i < cap; i += kRedBlock) {
        skey[i] = -1;
        sval[i] = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < f; i += kRedBlock) {
        const int2 p = pr[i];
        tbl_insert<int32_t>(skey, sval, cap - 1, lg, p.x, p.y);
    }
    __syncthreads();
    const int64_t cv = vweight(a.vwgt, hp.hubs[h]);
    unsigned long long best = 0;
    for (int i = threadIdx.x; i < cap; i += kRedBlock) {
        const int32_t L = skey[i];
        if (L >= 0 && a.W[L] + cv <= capof(a, L)) {
            const unsigned long long pk = pack_best(sval[i], L);
            best = pk > best ? pk : best;
        }
    }
    best = block_max<kRedBlock>(best, tmp);
    if (threadIdx.x == 0) {
        if (best) atomicMax(&hp.best[h], best);
        hp.fill[gb] = 0;
    }
}

// Overflow tables of the hubs flagged in ovf: best label with room over each
// slice, then the slice is emptied for the next round. Hubs without overflow
// cost one flag load per slice.
__global__ __launch_bounds__(256) void k_hub_scan(LPArgs a, HubPlan hp, int32_t nslices) {
    if (*a.done) return;
    __shared__ unsigned long long tmp[256 / kWave + 1];
    for (int32_t sl = blockIdx.x; sl < nslices; sl += gridDim.x) {
        const int32_t h = hp.slice_hub[sl];
        if (!hp.ovf[h]) continue;  // uniform
        const uint32_t tcap = 1u << hp.tlog[h];
        const uint32_t s0 = (uint32_t)(sl - hp.slice_first[h]) * kHubSlice;
        const uint32_t s1 = min(tcap, s0 + kHubSlice);
        int32_t *key = hp.key + hp.toff[h];
        int32_t *val = hp.val + hp.toff[h];
        const int64_t cv = vweight(a.vwgt, hp.hubs[h]);
        unsigned long long best = 0;
        for (uint32_t i = s0 + threadIdx.x; i < s1; i += 256) {
            const int32_t L = key[i];
            if (L >= 0) {
                if (a.W[L] + cv <= capof(a, L)) {
                    const unsigned long long pk = pack_best(val[i], L);
                    best = pk > best ? pk : best;
                }
                key[i] = -1;
                val[i] = 0;
            }
        }
        best = block_max<256>(best, tmp);
        if (threadIdx.x == 0 && best) atomicMax(&hp.best[h], best);
    }
}

// The hub proposes its best label with room if that connection beats the one
// to its own label (the same rule as the other tiers: the strongest eligible
// label, ties to the smaller label); resets the per-hub state.
__global__ void k_hub_decide(LPArgs a, HubPlan hp, int32_t nh) {
    if (*a.done) return;
    for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
        const int64_t oc = (int64_t)hp.own[h];
        const unsigned long long b = hp.best[h];
        int32_t target = -1;
        if (b) {
            const int64_t c = (int64_t)(b >> 32);
            const int32_t L = INT_MAX - (int32_t)(uint32_t)(b & 0xFFFFFFFFull);
            if (c > oc) target = L;
        }
        a.prop[hp.hubs[h]] = target;
        hp.own[h] = 0;
        hp.best[h] = 0;
        hp.ovf[h] = 0;
    }
}

__global__ void k_hub_plan(const int32_t *xadj, const int32_t *hubs, int32_t nh, int32_t *tlog, int64_t *tcap,
                           int32_t *nchunk, int32_t *nslice, int32_t *nbk) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = hubs[i];
        const int64_t d = xadj[v + 1] - xadj[v];
        int lg = 1;
        while ((int64_t(1) << lg) < 2 * d) lg++;
        tlog[i] = lg;
        tcap[i] = int64_t(1) << lg;
        nchunk[i] = (int32_t)((d + kHubChunk - 1) / kHubChunk);
        nslice[i] = (int32_t)(((int64_t(1) << lg) + kHubSlice - 1) / kHubSlice);
        nbk[i] = (int32_t)min<int64_t>(max<int64_t>((d + kHubPer - 1) / kHubPer, 1), kHubMaxBuck);
    }
}

__global__ void k_hub_expand(const int32_t *first, const int32_t *num, int32_t nh, int32_t *owner) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t j = 0; j < num[i]; j++) owner[first[i] + j] = (int32_t)i;
}

// ---------------------------------------------------------------- dense tables (few labels)

// Refinement of a k-way partition: labels are block ids < nlabels <= KT, so
// the per-vertex table is a dense array of KT connection sums (no hashing)
// and the k label weights of the round start sit in LDS, which lets the
// capacity test run inside the single selection pass. The first two GL-entry
// chunks of a group's next vertex (ids, weights, then labels) are loaded
// while the current vertex is selected, so each vertex's chain of dependent
// loads overlaps the previous vertex's reductions.
template <int GL, int KT, typename AccT>
__global__ __launch_bounds__(kPropBlock) void k_dense_group(LPArgs a, int32_t nlabels, TierList lists, int tier) {
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int GPW = kWave / GL;
    constexpr int NW = kPropBlock / kWave;
    // one table per lane group, KT + 1 apart so that the same block id of two
    // groups falls in different LDS banks
    __shared__ AccT sval[NW * GPW * (KT + 1)];
    __shared__ int64_t sW[KT];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int gl = lane % GL, grp = lane / GL;
    AccT *val = sval + (w * GPW + grp) * (KT + 1);
    // slack of each label at the round start: W - capacity (> 0 never eligible)
    for (int i = threadIdx.x; i < KT; i += kPropBlock) sW[i] = i < nlabels ? a.W[i] - capof(a, i) : (int64_t(1) << 62);
    for (int i = gl; i < KT; i += GL) val[i] = 0;
    __syncthreads();
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * NW * GPW;
    int64_t wb = ((int64_t)b * NW + w) * GPW;
    // the group's vertex and its first two chunks, loaded one iteration ahead
    bool valid = wb + grp < count;
    int32_t v = valid ? verts[wb + grp] : 0;
    int32_t beg = valid ? a.xadj[v] : 0;
    int32_t end = (valid && !inactive(a, v)) ? a.xadj[v + 1] : beg;
    int32_t own = valid ? a.labels[v] : -1;
    int32_t u0 = beg + gl < end ? a.adjncy[beg + gl] : -1, u1 = beg + gl + GL < end ? a.adjncy[beg + gl + GL] : -1;
    AccT w0 = (u0 >= 0 && a.adjwgt) ? (AccT)a.adjwgt[beg + gl] : (AccT)1;
    AccT w1 = (u1 >= 0 && a.adjwgt) ? (AccT)a.adjwgt[beg + gl + GL] : (AccT)1;
    int32_t L0 = u0 >= 0 ? (int32_t)a.lab8[u0] : -1, L1 = u1 >= 0 ? (int32_t)a.lab8[u1] : -1;
    for (; wb < count; wb += stride) {
        const int64_t nwb = wb + stride;
        const bool nvalid = nwb + grp < count;
        const int32_t nv = nvalid ? verts[nwb + grp] : 0;
        AccT oc = 0;
        const int nch = (end - beg + GL - 1) / GL;
        const int maxch = wave_max(nch);
        // chunks 0 and 1 from the registers, the rest as they come
        if (u0 >= 0) {
            if (L0 == own) oc += w0;
            else if (dir_ok(L0, own, dmode)) lds_add<AccT>(&val[L0], w0);
        }
        if (u1 >= 0) {
            if (L1 == own) oc += w1;
            else if (dir_ok(L1, own, dmode)) lds_add<AccT>(&val[L1], w1);
        }
        for (int ch = 2; ch < maxch; ch += 2) {
            const int32_t e0 = beg + ch * GL + gl, e1 = e0 + GL;
            const int32_t x0 = e0 < end ? a.adjncy[e0] : -1, x1 = e1 < end ? a.adjncy[e1] : -1;
            const AccT y0 = (e0 < end && a.adjwgt) ? (AccT)a.adjwgt[e0] : (AccT)1;
            const AccT y1 = (e1 < end && a.adjwgt) ? (AccT)a.adjwgt[e1] : (AccT)1;
            const int32_t M0 = x0 >= 0 ? (int32_t)a.lab8[x0] : -1, M1 = x1 >= 0 ? (int32_t)a.lab8[x1] : -1;
            if (x0 >= 0) {
                if (M0 == own) oc += y0;
                else if (dir_ok(M0, own, dmode)) lds_add<AccT>(&val[M0], y0);
            }
            if (x1 >= 0) {
                if (M1 == own) oc += y1;
                else if (dir_ok(M1, own, dmode)) lds_add<AccT>(&val[M1], y1);
            }
        }
        // the next vertex's row, label and first two chunks
        const int32_t nbeg = nvalid ? a.xadj[nv] : 0;
        const int32_t nend = (nvalid && !inactive(a, nv)) ? a.xadj[nv + 1] : nbeg;
        const int32_t nown = nvalid ? a.labels[nv] : -1;
        u0 = nbeg + gl < nend ? a.adjncy[nbeg + gl] : -1;
        u1 = nbeg + gl + GL < nend ? a.adjncy[nbeg + gl + GL] : -1;
        w0 = (u0 >= 0 && a.adjwgt) ? (AccT)a.adjwgt[nbeg + gl] : (AccT)1;
        w1 = (u1 >= 0 && a.adjwgt) ? (AccT)a.adjwgt[nbeg + gl + GL] : (AccT)1;
        wave_sync();
        oc = group_sum<GL>(oc);
        L0 = u0 >= 0 ? (int32_t)a.lab8[u0] : -1;
        L1 = u1 >= 0 ? (int32_t)a.lab8[u1] : -1;
        const int64_t cv = valid ? vweight(a.vwgt, v) : 0;
        AccT bc = 0;
        int32_t bl = INT_MAX;
        for (int i = gl; i < KT; i += GL) {
            const AccT c = val[i];
            if (c > 0 && sW[i] + cv <= 0 && better(c, i, bc, bl)) {
                bc = c;
                bl = i;
            }
        }
        group_best<GL, AccT>(bc, bl);
        if (valid && gl == 0) a.prop[v] = (bl != INT_MAX && bc > oc) ? bl : -1;
        wave_sync();
        for (int i = gl; i < KT; i += GL) val[i] = 0;
        wave_sync();
        valid = nvalid;
        v = nv;
        beg = nbeg;
        end = nend;
        own = nown;
    }
}

// Dense-table counterpart of k_plane for the tiers of at most E neighbours
// (4 or 8, E <= GL): one entry per lane, each label's connection summed over
// the group's first E lanes by shuffles, the k label weights of the round
// start in LDS, the rule of k_dense_group.
template <int GL, int E, int KT, typename AccT>
__global__ __launch_bounds__(kPropBlock) void k_dense_lanes(LPArgs a, int32_t nlabels, TierList lists, int tier) {
    static_assert(E <= GL, "one entry per lane");
    if (*a.done) return;
    const int64_t t0 = lists.ts[tier];
    const int32_t count = (int32_t)(lists.ts[tier + 1] - t0);
    const int32_t *__restrict__ verts = lists.verts + t0;
    const int32_t dmode = cur_dirmode(a);
    constexpr int GPW = kWave / GL;
    constexpr int NW = kPropBlock / kWave;
    __shared__ int64_t sW[KT];
    for (int i = threadIdx.x; i < KT; i += kPropBlock) sW[i] = i < nlabels ? a.W[i] - capof(a, i) : (int64_t(1) << 62);
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const int gl = lane % GL, grp = lane / GL;
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t stride = (int64_t)gridDim.x * NW * GPW;
    int64_t wb = ((int64_t)b * NW + w) * GPW;
    bool valid = wb + grp < count;
    int32_t v = valid ? verts[wb + grp] : 0;
    int32_t beg = valid ? a.xadj[v] : 0;
    int32_t end = (valid && !inactive(a, v)) ? a.xadj[v + 1] : beg;
    int32_t own = valid ? a.labels[v] : -1;
    int32_t u = beg + gl < end ? a.adjncy[beg + gl] : -1;
    AccT wt = (u >= 0 && a.adjwgt) ? (AccT)a.adjwgt[beg + gl] : (AccT)1;
    int32_t L = u >= 0 ? (int32_t)a.lab8[u] : -1;
    for (; wb < count; wb += stride) {
        const int64_t nwb = wb + stride;
        const bool nvalid = nwb + grp < count;
        const int32_t nv = nvalid ? verts[nwb + grp] : 0;
        const int32_t nbeg = nvalid ? a.xadj[nv] : 0;
        const int32_t nend = (nvalid && !inactive(a, nv)) ? a.xadj[nv + 1] : nbeg;
        const int32_t nown = nvalid ? a.labels[nv] : -1;
        const int32_t nu = nbeg + gl < nend ? a.adjncy[nbeg + gl] : -1;
        const AccT nwt = (nu >= 0 && a.adjwgt) ? (AccT)a.adjwgt[nbeg + gl] : (AccT)1;
        AccT c = 0;
#pragma unroll
        for (int d = 0; d < E; d++) {
            const int32_t Ld = __shfl(L, d, GL);
            const AccT wd = __shfl(wt, d, GL);
            if (Ld == L) c += wd;
        }
        const AccT oc = group_sum<GL>((L >= 0 && L == own) ? wt : (AccT)0);
        const int64_t cv = valid ? vweight(a.vwgt, v) : 0;
        AccT bc = 0;
        int32_t bl = INT_MAX;
        if (L >= 0 && L != own && c > 0 && dir_ok(L, own, dmode) && sW[L] + cv <= 0) {
            bc = c;
            bl = L;
        }
        group_best<GL, AccT>(bc, bl);
        if (valid && gl == 0) a.prop[v] = (bl != INT_MAX && bc > oc) ? bl : -1;
        valid = nvalid;
        v = nv;
        own = nown;
        u = nu;
        wt = nwt;
        L = nu >= 0 ? (int32_t)a.lab8[nu] : -1;
    }
}

// Vertices above the group tiers in dense mode: edges cut into chunks of
// kDenseChunk entries, one workgroup per chunk; each chunk adds its k
// connection sums into the vertex's row of a global [nbig x KT] array, then
// one wave per vertex selects. No single workgroup walks a whole hub.
struct DenseBig {
    const int32_t *verts;        // [nbig]
    const int4 *desc;            // [nchunks] (vertex, first entry, end entry, index into verts)
    void *gconn;                 // [nbig * KT] AccT
    unsigned long long *own;     // [nbig]
    int32_t nbig;
    int32_t chunk;               // entries per chunk workgroup
};

template <typename AccT>
__device__ __forceinline__ void gadd(AccT *p, AccT w);
template <>
__device__ __forceinline__ void gadd<int32_t>(int32_t *p, int32_t w) {
    atomicAdd(p, w);
}
template <>
__device__ __forceinline__ void gadd<int64_t>(int64_t *p, int64_t w) {
    atomicAdd((unsigned long long *)p, (unsigned long long)w);
}

template <int KT, typename AccT>
__global__ __launch_bounds__(256) void k_dense_chunk(LPArgs a, DenseBig db) {
    if (*a.done) return;
    const int32_t dmode = cur_dirmode(a);
    constexpr int NW = 256 / kWave;
    // SUB tables per wave (lanes split evenly) spread the LDS atomics of a
    // wave over SUB x KT addresses when k is small
    constexpr int SUB = KT <= 64 ? 8 : 2;
    // rows KT + 1 apart: the same block id of two tables falls in different LDS banks
    __shared__ AccT val[NW * SUB][KT + 1];
    __shared__ AccT tmp[NW + 1];
    const int w = (threadIdx.x / kWave) * SUB + lane_id() / (kWave / SUB);
    for (int i = threadIdx.x; i < NW * SUB * (KT + 1); i += 256) (&val[0][0])[i] = 0;
    __syncthreads();
    // the chunk's vertex and entry range come in one load (planned once per
    // call), so the edge loads wait on one load, not on three dependent ones
    const int4 d = db.desc[blockIdx.x];
    const int32_t v = d.x, beg = d.y, b = d.w;
    if (inactive(a, v)) return;  // uniform: the vertex's row stays zero
    const int32_t end = d.z;
    const int32_t own = a.labels[v];
    AccT oc = 0;
    constexpr int UC = 4;
    for (int32_t e0 = beg + threadIdx.x; e0 < end; e0 += UC * 256) {
        int32_t u[UC], L[UC];
        AccT wv[UC];
#pragma unroll
        for (int j = 0; j < UC; j++) {
            const int32_t e = e0 + j * 256;
            u[j] = e < end ? a.adjncy[e] : -1;
            wv[j] = (e < end && a.adjwgt) ? (AccT)a.adjwgt[e] : (AccT)1;
        }
#pragma unroll
        for (int j = 0; j < UC; j++) L[j] = u[j] >= 0 ? (int32_t)a.lab8[u[j]] : -1;
#pragma unroll
        for (int j = 0; j < UC; j++) {
            if (u[j] < 0) continue;
            if (L[j] == own) oc += wv[j];
            else if (dir_ok(L[j], own, dmode)) lds_add<AccT>(&val[w][L[j]], wv[j]);
        }
    }
    __syncthreads();
    AccT *row = (AccT *)db.gconn + (int64_t)b * KT;
    // all threads reduce the tables: P consecutive lanes per block id
    constexpr int P = 256 / KT, NT = NW * SUB;
    const int lab = threadIdx.x / P, part = threadIdx.x % P;
    AccT c = 0;
    for (int q = part; q < NT; q += P) c += val[q][lab];
    c = group_sum<P>(c);
    if (part == 0 && c) gadd<AccT>(&row[lab], c);
    oc = block_sum<256>(oc, tmp);
    if (threadIdx.x == 0 && oc) atomicAdd(&db.own[b], (unsigned long long)oc);
}

template <int KT, typename AccT>
__global__ __launch_bounds__(256) void k_dense_finish(LPArgs a, DenseBig db, int32_t nlabels) {
    if (*a.done) return;
    const int32_t dmode = cur_dirmode(a);
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int32_t b = blockIdx.x * (256 / kWave) + w;
    if (b >= db.nbig) return;
    const int32_t v = db.verts[b];
    AccT *row = (AccT *)db.gconn + (int64_t)b * KT;
    const int64_t cv = vweight(a.vwgt, v);
    const int64_t oc = (int64_t)db.own[b];
    AccT bc = 0;
    int32_t bl = INT_MAX;
    for (int i = lane; i < nlabels; i += kWave) {
        const AccT c = row[i];
        if (c > 0 && a.W[i] + cv <= capof(a, i) && better(c, i, bc, bl)) {
            bc = c;
            bl = i;
        }
        row[i] = 0;
    }
    group_best<kWave, AccT>(bc, bl);
    if (lane == 0) {
        a.prop[v] = (bl != INT_MAX && (int64_t)bc > oc) ? bl : -1;
        db.own[b] = 0;
    }
}

template <int KT, typename AccT>
int launch_dense(const LPArgs &a, int32_t nlabels, const int64_t *tstart, TierList tl, const DenseBig *db,
                 int32_t nchunks, hipStream_t s, const double *tb, int tg_end) {
    const std::string sfx = std::string(", ") + std::to_string(KT) + ", " + (sizeof(AccT) == 4 ? "int" : "long") + ">";
    // grids are sized by the full tier (an upper bound of the list the kernel reads)
    // tiers from tg_end on read connection rows instead
    auto cnt = [&](int t) { return t < tg_end ? (int32_t)(tstart[t + 1] - tstart[t]) : 0; };
    constexpr int NW = kPropBlock / kWave;
    constexpr int G1 = KT >= 256 ? 16 : 4;
    constexpr int G2 = KT >= 256 ? 16 : 8;
    auto blocks_for = [&](int32_t c, int per_block) { return grid_for(c, per_block, 16384); };
    int32_t c;
    if ((c = cnt(1)) > 0)
        GP_PROF_LAUNCH((std::string("k_dense_lanes<") + std::to_string(G1) + sfx).c_str(), tb[1], s, hipLaunchKernelGGL((k_dense_lanes<G1, 4, KT, AccT>), dim3(blocks_for(c, NW * (kWave / G1))), dim3(kPropBlock), 0,
                           s, a, nlabels, tl, 1));
    if ((c = cnt(2)) > 0)
        GP_PROF_LAUNCH((std::string("k_dense_lanes<") + std::to_string(G2) + sfx).c_str(), tb[2], s, hipLaunchKernelGGL((k_dense_lanes<G2, 8, KT, AccT>), dim3(blocks_for(c, NW * (kWave / G2))), dim3(kPropBlock), 0,
                           s, a, nlabels, tl, 2));
    if ((c = cnt(3)) > 0)
        GP_PROF_LAUNCH((std::string("k_dense_group<16") + sfx).c_str(), tb[3], s, hipLaunchKernelGGL((k_dense_group<16, KT, AccT>), dim3(blocks_for(c, NW * 4)), dim3(kPropBlock), 0, s, a,
                           nlabels, tl, 3));
    if ((c = cnt(4)) > 0)
        GP_PROF_LAUNCH((std::string("k_dense_group<32") + sfx).c_str(), tb[4], s, hipLaunchKernelGGL((k_dense_group<32, KT, AccT>), dim3(blocks_for(c, NW * 2)), dim3(kPropBlock), 0, s, a,
                           nlabels, tl, 4));
    if ((c = cnt(5)) > 0)
        GP_PROF_LAUNCH((std::string("k_dense_group<64") + sfx).c_str(), tb[5], s, hipLaunchKernelGGL((k_dense_group<64, KT, AccT>), dim3(blocks_for(c, NW)), dim3(kPropBlock), 0, s, a, nlabels,
                           tl, 5));
    if (db && db->nbig > 0) {
        GP_PROF_LAUNCH((std::string("k_dense_chunk<") + std::to_string(KT) + sfx.substr(std::to_string(KT).size() + 2)).c_str(), tb[6] + tb[7] + tb[8] + tb[9] + tb[10], s, hipLaunchKernelGGL((k_dense_chunk<KT, AccT>), dim3(nchunks), dim3(256), 0, s, a, *db));
        hipLaunchKernelGGL((k_dense_finish<KT, AccT>), dim3((db->nbig + 3) / 4), dim3(256), 0, s, a, *db, nlabels);
    }
    GP_LAUNCH_CHECK();
    return GP_OK;
}

template <typename AccT>
int launch_dense_any(const LPArgs &a, int32_t nlabels, const int64_t *tstart, TierList tl, const DenseBig *db,
                     int32_t nchunks, hipStream_t s, const double *tb, int tg_end) {
    if (nlabels <= 16) return launch_dense<16, AccT>(a, nlabels, tstart, tl, db, nchunks, s, tb, tg_end);
    if (nlabels <= 64) return launch_dense<64, AccT>(a, nlabels, tstart, tl, db, nchunks, s, tb, tg_end);
    return launch_dense<256, AccT>(a, nlabels, tstart, tl, db, nchunks, s, tb, tg_end);
}

// ---------------------------------------------------------------- connection rows (refinement)
//
// Refinement rounds move few vertices (well under one percent of them per
// round on large graphs), yet a plain round gathers the neighbour labels of
// every vertex again. For the vertices above KT/8 neighbours the sums are
// therefore kept from round to round: row r holds the KT connection sums of
// table vertex r (own block included, no direction filter), filled once from
// the labels of the first round's start and afterwards changed only by the
// admitted moves. A vertex u moved from block a to block b takes the weight of
// each edge (u, v) off row(v)[a] and adds it to row(v)[b]; the edge lists are
// symmetric (§II-A), so the weight is found in u's own list. A round's
// proposal for a table vertex then reads KT sums instead of deg label gathers.
// The sums are integers: after every round the rows equal a recomputation
// from the labels, so the proposals are those of the plain rounds.

// Rows of table vertices 0 .. count-1 (tverts) from the labels: one wave per
// vertex, a KT-sum LDS table per wave, written out whole.
template <int KT, typename AccT>
__global__ __launch_bounds__(256) void k_rows_fill(const int32_t *__restrict__ xadj, const int32_t *__restrict__ adjncy,
                                                   const int32_t *__restrict__ adjwgt, const uint8_t *__restrict__ lab8,
                                                   const int32_t *__restrict__ tverts, int32_t count, AccT *rows) {
    constexpr int NW = 256 / kWave;
    __shared__ AccT sval[NW][KT + 1];
    const int w = threadIdx.x / kWave, lane = lane_id();
    AccT *val = sval[w];
    for (int i = lane; i < KT; i += kWave) val[i] = 0;
    wave_sync();
    for (int64_t j = (int64_t)blockIdx.x * NW + w; j < count; j += (int64_t)gridDim.x * NW) {
        const int32_t v = tverts[j];
        const int32_t beg = xadj[v], end = xadj[v + 1];
        for (int32_t e = beg + lane; e < end; e += kWave)
            lds_add<AccT>(&val[lab8[adjncy[e]]], adjwgt ? (AccT)adjwgt[e] : (AccT)1);
        wave_sync();
        AccT *row = rows + j * KT;
        for (int i = lane; i < KT; i += kWave) {
            row[i] = val[i];
            val[i] = 0;
        }
        wave_sync();
    }
}

// Rows of the chunked big vertices: chunk (vertex, first entry, end entry, b)
// adds its sums into row rowbase + b, which starts at zero.
template <int KT, typename AccT>
__global__ __launch_bounds__(256) void k_rows_fill_chunk(const int32_t *__restrict__ adjncy,
                                                         const int32_t *__restrict__ adjwgt,
                                                         const uint8_t *__restrict__ lab8, const int4 *desc,
                                                         int32_t rowbase, AccT *rows) {
    constexpr int NW = 256 / kWave;
    constexpr int SUB = KT <= 64 ? 8 : 2;
    __shared__ AccT val[NW * SUB][KT + 1];
    const int w = (threadIdx.x / kWave) * SUB + lane_id() / (kWave / SUB);
    for (int i = threadIdx.x; i < NW * SUB * (KT + 1); i += 256) (&val[0][0])[i] = 0;
    __syncthreads();
    const int4 d = desc[blockIdx.x];
    constexpr int UC = 4;
    for (int32_t e0 = d.y + threadIdx.x; e0 < d.z; e0 += UC * 256) {
        int32_t u[UC];
        AccT wv[UC];
#pragma unroll
        for (int q = 0; q < UC; q++) {
            const int32_t e = e0 + q * 256;
            u[q] = e < d.z ? adjncy[e] : -1;
            wv[q] = (e < d.z && adjwgt) ? (AccT)adjwgt[e] : (AccT)1;
        }
#pragma unroll
        for (int q = 0; q < UC; q++)
            if (u[q] >= 0) lds_add<AccT>(&val[w][lab8[u[q]]], wv[q]);
    }
    __syncthreads();
    AccT *row = rows + (int64_t)(rowbase + d.w) * KT;
    constexpr int P = 256 / KT, NT = NW * SUB;
    const int lab = threadIdx.x / P, part = threadIdx.x % P;
    AccT c = 0;
    for (int q = part; q < NT; q += P) c += val[q][lab];
    c = group_sum<P>(c);
    if (part == 0 && c) gadd<AccT>(&row[lab], c);
}

// Four consecutive sums of a row in 16-byte loads.
template <typename AccT>
__device__ __forceinline__ void load4(const AccT *p, AccT (&c)[4]);
template <>
__device__ __forceinline__ void load4<int32_t>(const int32_t *p, int32_t (&c)[4]) {
    const int4 x = *reinterpret_cast<const int4 *>(p);
    c[0] = x.x;
    c[1] = x.y;
    c[2] = x.z;
    c[3] = x.w;
}
template <>
__device__ __forceinline__ void load4<int64_t>(const int64_t *p, int64_t (&c)[4]) {
    const longlong2 x = reinterpret_cast<const longlong2 *>(p)[0], y = reinterpret_cast<const longlong2 *>(p)[1];
    c[0] = x.x;
    c[1] = x.y;
    c[2] = y.x;
    c[3] = y.y;
}

// A round's proposals of the table vertices (list entries ts[tfirst] ..
// ts[tend]): KT/4 lanes per vertex read its row, four sums per lane, and the
// rule of the other kernels is applied to the sums (strongest eligible block
// other than its own, ties to the smaller id, taken if it beats the own
// block's sum). Each lane group has UV vertices in flight. Entry j of the full
// list is row j; the per-round lists of active-set rounds look the row up in
// rowidx. Also empties the round's queue of big movers.
template <int KT, typename AccT>
__global__ __launch_bounds__(kPropBlock) void k_dense_rows(LPArgs a, int32_t nlabels, TierList lists, int tfirst,
                                                           int tend, const AccT *__restrict__ rows,
                                                           const int32_t *__restrict__ rowidx, int32_t *nbig) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *nbig = 0;
    if (*a.done) return;
    constexpr int GL = KT / 4;
    constexpr int GPW = kWave / GL;
    constexpr int NW = kPropBlock / kWave;
    constexpr int UV = 4;
    __shared__ int64_t sW[KT];
    for (int i = threadIdx.x; i < KT; i += kPropBlock) sW[i] = i < nlabels ? a.W[i] - capof(a, i) : (int64_t(1) << 62);
    __syncthreads();
    const int64_t t0 = lists.ts[tfirst];
    const int64_t count = lists.ts[tend] - t0;
    const int32_t dmode = cur_dirmode(a);
    const int lane = lane_id(), gl = lane % GL, grp = lane / GL, w = threadIdx.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * NW * GPW;
    for (int64_t base = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * NW + w) * GPW + grp; base - grp < count;
         base += UV * stride) {
        int32_t v[UV], own[UV];
        bool valid[UV], live[UV];
        AccT c[UV][4];
#pragma unroll
        for (int u = 0; u < UV; u++) {
            const int64_t j = base + u * stride;
            valid[u] = j < count;
            v[u] = valid[u] ? lists.verts[t0 + j] : 0;
            if (!rowidx && valid[u]) load4<AccT>(rows + j * KT + 4 * gl, c[u]);
        }
#pragma unroll
        for (int u = 0; u < UV; u++) {
            live[u] = valid[u] && !inactive(a, v[u]);
            own[u] = live[u] ? a.labels[v[u]] : -1;
            if (rowidx && valid[u]) load4<AccT>(rows + (int64_t)rowidx[v[u]] * KT + 4 * gl, c[u]);
        }
#pragma unroll
        for (int u = 0; u < UV; u++) {
            const int64_t cv = live[u] ? vweight(a.vwgt, v[u]) : 0;
            AccT oc = 0, bc = 0;
            int32_t bl = INT_MAX;
            if (live[u]) {
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int32_t i = 4 * gl + q;
                    const AccT x = c[u][q];
                    if (i == own[u]) oc = x;
                    else if (x > 0 && dir_ok(i, own[u], dmode) && sW[i] + cv <= 0 && better(x, i, bc, bl)) {
                        bc = x;
                        bl = i;
                    }
                }
            }
            oc = group_sum<GL>(oc);
            group_best<GL, AccT>(bc, bl);
            if (valid[u] && gl == 0) a.prop[v[u]] = (bl != INT_MAX && bc > oc) ? bl : -1;
        }
    }
}

// After the admission: the admitted movers' edges change the rows of their
// table neighbours. 16 lanes per mover; a mover above kRowSplit neighbours is
// queued instead as chunks of kRowChunk entries (vertex, first entry, old
// block, new block), which k_rows_update_big spreads over whole workgroups.
constexpr int kRowSplit = 256;
constexpr int kRowChunk = 4096;
template <typename AccT>
__device__ __forceinline__ void row_move(AccT *rows, int KT, int32_t r, int32_t from, int32_t to, AccT w) {
    AccT *row = rows + (int64_t)r * KT;
    gadd<AccT>(&row[from], (AccT)-w);
    gadd<AccT>(&row[to], w);
}

template <int KT, typename AccT>
__global__ __launch_bounds__(256) void k_rows_update(const uint32_t *mk, const int32_t *mv, const int32_t *oldlab,
                                                     const int32_t *nmov, const int32_t *__restrict__ xadj,
                                                     const int32_t *__restrict__ adjncy,
                                                     const int32_t *__restrict__ adjwgt,
                                                     const int32_t *__restrict__ rowidx, AccT *rows, int4 *big,
                                                     int32_t *nbig, unsigned long long *pushed_total) {
    constexpr int GL = 16;
    const int32_t n = *nmov;
    const int gl = threadIdx.x % GL;
    const int64_t step = (int64_t)gridDim.x * blockDim.x / GL;
    long long pushed = 0;  // the movers' edges, counted once per mover
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GL; p < n; p += step) {
        const int32_t from = oldlab[p];
        if (from < 0) continue;  // refused by the admission
        const int32_t u = mv[p], to = (int32_t)mk[p];
        const int32_t e0 = xadj[u], e1 = xadj[u + 1];
        if (gl == 0) pushed += e1 - e0;
        if (e1 - e0 > kRowSplit) {
            if (gl == 0) {
                const int32_t nc = (e1 - e0 + kRowChunk - 1) / kRowChunk;
                const int32_t at = atomicAdd(nbig, nc);
                for (int32_t q = 0; q < nc; q++) big[at + q] = make_int4(u, e0 + q * kRowChunk, from, to);
            }
            continue;
        }
        for (int32_t e = e0 + gl; e < e1; e += GL) {
            const int32_t r = rowidx[adjncy[e]];
            if (r >= 0) row_move<AccT>(rows, KT, r, from, to, adjwgt ? (AccT)adjwgt[e] : (AccT)1);
        }
    }
    pushed = wave_sum(pushed);
    if (lane_id() == 0 && pushed) atomicAdd(pushed_total, (unsigned long long)pushed);
}

template <int KT, typename AccT>
__global__ __launch_bounds__(256) void k_rows_update_big(const int4 *big, const int32_t *nbig,
                                                         const int32_t *__restrict__ xadj,
                                                         const int32_t *__restrict__ adjncy,
                                                         const int32_t *__restrict__ adjwgt,
                                                         const int32_t *__restrict__ rowidx, AccT *rows) {
    const int32_t nb = *nbig;
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int4 c = big[i];
        const int32_t e1 = min(xadj[c.x + 1], c.y + kRowChunk);
        for (int32_t e = c.y + threadIdx.x; e < e1; e += 256) {
            const int32_t r = rowidx[adjncy[e]];
            if (r >= 0) row_move<AccT>(rows, KT, r, c.z, c.w, adjwgt ? (AccT)adjwgt[e] : (AccT)1);
        }
    }
}

// rowidx[v] = row of table vertex v (list entry first + j holds row j)
__global__ void k_rows_index(const int32_t *verts, int64_t first, int32_t nt, int32_t *rowidx) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nt; j += (int64_t)gridDim.x * blockDim.x)
        rowidx[verts[first + j]] = (int32_t)j;
}

// Connection rows of one LP run (rows == nullptr: plain rounds). Table
// vertices are the tier-list entries from tier tfirst on; row j belongs to
// entry tstart[tfirst] + j.
struct RowTables {
    void *rows = nullptr;     // [nt * KT] AccT
    int32_t *rowidx = nullptr;  // [n] row of each vertex, -1 outside the table
    int4 *big = nullptr;      // the round's chunks of movers above kRowSplit neighbours
    int32_t *nbig = nullptr;
    int tfirst = 0;
    int32_t nt = 0;
    int32_t nsmall = 0;  // rows filled per vertex; the rest (chunked big vertices) by chunks
    int64_t entries = 0;  // edges of the table vertices
    unsigned long long *pushed = nullptr;  // edges of the admitted movers pushed into rows
    double sel_bytes = 0;
};

template <int KT, typename AccT>
int rows_fill(const RowTables &rt, const int32_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
              const uint8_t *lab8, const int32_t *tverts, const DenseBig *db, int32_t nchunks, hipStream_t s) {
    if (rt.nsmall > 0)
        hipLaunchKernelGGL((k_rows_fill<KT, AccT>), dim3(grid_for(rt.nsmall, 256 / kWave, 16384)), dim3(256), 0, s,
                           xadj, adjncy, adjwgt, lab8, tverts, rt.nsmall, (AccT *)rt.rows);
    if (db && db->nbig > 0 && nchunks > 0)
        hipLaunchKernelGGL((k_rows_fill_chunk<KT, AccT>), dim3(nchunks), dim3(256), 0, s, adjncy, adjwgt, lab8,
                           db->desc, rt.nsmall, (AccT *)rt.rows);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

template <int KT, typename AccT>
int rows_select(const LPArgs &a, int32_t nlabels, TierList tl, const RowTables &rt, int tend, bool active,
                hipStream_t s) {
    constexpr int per_block = (kPropBlock / kWave) * (kWave / (KT / 4)) * 4;
    const std::string name = std::string("k_dense_rows<") + std::to_string(KT) + (sizeof(AccT) == 4 ? ", int>" : ", long>");
    GP_PROF_LAUNCH(name.c_str(), rt.sel_bytes, s, hipLaunchKernelGGL((k_dense_rows<KT, AccT>), dim3(grid_for(rt.nt, per_block, 16384)), dim3(kPropBlock), 0, s, a, nlabels, tl, rt.tfirst, tend, (const AccT *)rt.rows, active ? rt.rowidx : nullptr, rt.nbig));
    GP_LAUNCH_CHECK();
    return GP_OK;
}

template <int KT, typename AccT>
int rows_update(const RowTables &rt, const uint32_t *mk, const int32_t *mv, const int32_t *oldlab,
                const int32_t *nmov, const int32_t *xadj, const int32_t *adjncy, const int32_t *adjwgt, int64_t n,
                int64_t nnz, hipStream_t s) {
    hipLaunchKernelGGL((k_rows_update<KT, AccT>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, mk, mv, oldlab, nmov,
                       xadj, adjncy, adjwgt, rt.rowidx, (AccT *)rt.rows, rt.big, rt.nbig, rt.pushed);
    hipLaunchKernelGGL((k_rows_update_big<KT, AccT>), dim3(grid_for(nnz / kRowChunk + 1, 1, 4096)), dim3(256), 0, s,
                       rt.big, rt.nbig, xadj, adjncy, adjwgt, rt.rowidx, (AccT *)rt.rows);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

// GP_REFINE_ROWS=0 runs every refinement round on label gathers; unset or any
// other value keeps connection rows where they are allowed. Read at every LP run.
bool use_refine_rows() {
    const char *e = std::getenv("GP_REFINE_ROWS");
    return !(e && std::strcmp(e, "0") == 0);
}
// largest row storage of one LP run
constexpr double kRowsMaxBytes = 32.0 * (1 << 30);

__global__ void k_labels_u8(const int32_t *labels, int32_t n, uint8_t *lab8) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        lab8[v] = (uint8_t)labels[v];
}

__global__ void k_chunk_counts(const int32_t *xadj, const int32_t *verts, int32_t nb, int32_t chunk, int32_t *num) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = verts[i];
        num[i] = (xadj[v + 1] - xadj[v] + chunk - 1) / chunk;
    }
}

// chunk descriptors of the dense big-vertex plan: chunk q of vertex verts[i]
// covers entries [xadj[v] + q * chunk, min(xadj[v + 1], that + chunk))
__global__ void k_chunk_desc(const int32_t *xadj, const int32_t *verts, const int32_t *first, const int32_t *num,
                             int32_t nb, int32_t chunk, int4 *desc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = verts[i], e1 = xadj[v + 1];
        for (int32_t q = 0; q < num[i]; q++) {
            const int32_t b0 = xadj[v] + q * chunk;
            desc[first[i] + q] = make_int4(v, b0, min(e1, b0 + chunk), (int32_t)i);
        }
    }
}

// ---------------------------------------------------------------- tiers

// Degree tiers. Tier 0: no neighbours (never proposes). Tiers 1..5: GL lanes
// per vertex. Tiers 6..9: one workgroup per vertex (128, 256, 512 and 1024
// threads; the smaller ones fit more workgroups per CU). Tier 8's 64 KB packed
// table lets two of its workgroups share a CU, so one waits at a barrier while
// the other works; tier 9's 128 KB table takes a CU whole. Tier 10: hub
// (global table).
constexpr int kTiers = 11;

// Largest degree each hashed-table tier can hold (its table has 2x slots);
// the tuned bounds may only be lower.
__host__ __device__ inline int32_t tier_cap(int t, bool wide) {
    switch (t) {
        case 0: return 0;
        case 1: return 4;
        case 2: return 8;
        case 3: return 16;
        case 4: return 64;
        case 5: return 256;
        case 6: return 1024;
        case 7: return 2048;
        case 8: return 4096;
        case 9: return wide ? 4096 : 8192;
        default: return INT_MAX;
    }
}

struct TierKey {
    const int32_t *xadj;
    const int32_t *active;  // optional: labels array, vertices with label < 0 go to tier 0
    const uint8_t *frozen;  // optional: vertices with frozen[v] != 0 go to tier 0 (keep their label)
    bool wide;
    int32_t bound[kTiers];  // upper degree bound of each tier (non-decreasing, the last is INT_MAX)
};

__global__ void k_tier_keys(TierKey tk, int32_t n, uint32_t *key, int32_t *val, int32_t *counts,
                            unsigned long long *edges) {
    __shared__ int32_t h[kTiers];
    __shared__ unsigned long long he[kTiers];
    if (threadIdx.x < kTiers) {
        h[threadIdx.x] = 0;
        he[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = tk.xadj[v + 1] - tk.xadj[v];
        int t = 0;
        if (d > 0 && !(tk.active && tk.active[v] < 0) && !(tk.frozen && tk.frozen[v])) {
            t = 1;
            while (t < kTiers - 1 && d > tk.bound[t]) t++;
        }
        key[v] = (uint32_t)t;
        val[v] = (int32_t)v;
        atomicAdd(&h[t], 1);
        atomicAdd(&he[t], (unsigned long long)d);
    }
    __syncthreads();
    if (threadIdx.x < kTiers && h[threadIdx.x]) {
        atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
        atomicAdd(&edges[threadIdx.x], he[threadIdx.x]);
    }
}

__global__ void k_hub_caps(const int32_t *xadj, const int32_t *hubs, int32_t nh, int32_t *hlog,
                           int64_t *hcap) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = hubs[i];
        const int64_t d = xadj[v + 1] - xadj[v];
        int lg = 1;
        while ((int64_t(1) << lg) < 2 * d) lg++;
        hlog[i] = lg;
        hcap[i] = int64_t(1) << lg;
    }
}

// ---------------------------------------------------------------- admission / apply

struct MoverFlag {
    const int32_t *prop;
    const int32_t *done;
    __device__ bool operator()(int64_t i) const { return !*done && prop[i] >= 0; }
};
struct MoverEmit {
    const int32_t *prop;
    uint32_t *mk;
    int32_t *mv;
    __device__ void operator()(int64_t i, int32_t pos) const {
        mk[pos] = (uint32_t)prop[i];
        mv[pos] = (int32_t)i;
    }
};

struct MoverWeight {
    const int32_t *mv;
    const int32_t *vwgt;
    __device__ int64_t operator()(int64_t p) const { return vweight(vwgt, mv[p]); }
};
struct StoreIncl {
    int64_t *S;
    __device__ void operator()(int64_t p, int64_t ex, int64_t v) const { S[p] = ex + v; }
};


__global__ void k_heads(const uint32_t *mk, const int32_t *nmov, int32_t *headpos) {
    const int32_t n = *nmov;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        if (p == 0 || mk[p] != mk[p - 1]) headpos[mk[p]] = (int32_t)p;
}

__global__ void k_admit(const uint32_t *mk, const int32_t *mv, const int32_t *nmov, const int32_t *headpos,
                        const int64_t *S, const int64_t *W, int64_t U, const int64_t *capv, int32_t *labels,
                        uint8_t *lab8, int32_t *oldlab, LPDev *dev, const int32_t *group, GroupState *gs,
                        uint8_t *act) {
    const int32_t n = *nmov;
    const int lane = lane_id();
    int32_t cnt = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p - lane < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        bool moved = false;
        int32_t gq = 0;
        if (p < n) {
            const int32_t t = (int32_t)mk[p];
            const int32_t h = headpos[t];
            const int64_t pre = S[p] - (h > 0 ? S[h - 1] : 0);
            if (W[t] + pre <= (capv ? capv[t] : U)) {
                const int32_t v = mv[p];
                oldlab[p] = labels[v];
                labels[v] = t;
                if (lab8) lab8[v] = (uint8_t)t;
                cnt++;
                moved = true;
                if (group) gq = group[v];
            } else {
                oldlab[p] = -1;
                if (act && act[mv[p]] == 0) act[mv[p]] = 1;  // refused by capacity: evaluated again
            }
        }
        // movers sorted by target lie mostly in one graph: one count per wave
        const uint64_t mm = group ? __ballot(moved) : 0ull;
        if (mm) {
            const int32_t g0 = __shfl(gq, __ffsll((unsigned long long)mm) - 1, kWave);
            if (__ballot(moved && gq != g0) == 0) {
                if (lane == 0) atomicAdd(&gs[g0].moves, (int32_t)__popcll(mm));
            } else if (moved) {
                atomicAdd(&gs[gq].moves, 1);
            }
        }
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && cnt) atomicAdd(&dev->round_moves, cnt);
}
__global__ void k_apply_w(const uint32_t *mk, const int32_t *mv, const int32_t *nmov, const int32_t *oldlab,
                          const int32_t *vwgt, const int32_t *headpos, const int64_t *S, int64_t *W) {
    const int32_t n = *nmov;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t old = oldlab[p];
        if (old < 0) continue;
        const unsigned long long c = (unsigned long long)vweight(vwgt, mv[p]);
        atomicAdd((unsigned long long *)&W[old], (unsigned long long)(-(long long)c));
        const uint32_t t = mk[p];
        const bool tail = (p + 1 == n) || mk[p + 1] != t || oldlab[p + 1] < 0;
        if (tail) {
            const int32_t h = headpos[t];
            const int64_t in = S[p] - (h > 0 ? S[h - 1] : 0);
            atomicAdd((unsigned long long *)&W[t], (unsigned long long)in);
        }
    }
}

// Everything of a round after the proposals, in one workgroup, for graphs of
// at most kFuseMax vertices (single graphs without active sets): compaction
// of the movers in ascending vertex order, the stable sort by target, the
// segmented prefix of mover weights per target, admission against the
// weights of the round start, the label and weight updates and the round
// bookkeeping — the work of compact, radix_sort, k_heads, the prefix scan,
// k_admit, k_apply_w and k_round_end. A mover is packed as
// (target << vbits) | vertex in LDS. Position p of a sequence belongs to wave
// p / kFuseWaveSpan, row (p % kFuseWaveSpan) / kWave, lane p % kWave, so the
// (wave, row, lane) order is the position order.
constexpr int kFuseBlock = 1024;
constexpr int kFuseWaves = kFuseBlock / kWave;
constexpr int kFuseRows = 16;
constexpr int kFuseWaveSpan = kFuseRows * kWave;
constexpr int kFuseMax = kFuseBlock * kFuseRows;
constexpr int kFuseLdsLabels = 1024;  // label weights held in LDS for the whole round

// Exclusive prefix of x over the workgroup in thread order; *total gets the
// sum. Every thread adds up the wave totals before its own wave.
template <typename T>
__device__ __forceinline__ T fuse_excl_scan(T x, T *tmp, T *total) {
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const T inc = wave_incl_scan(x);
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kFuseWaves; i++) {
        const T t = tmp[i];
        before += i < w ? t : T(0);
        all += t;
    }
    *total = all;
    __syncthreads();
    return before + inc - x;
}

__global__ __launch_bounds__(kFuseBlock) void k_round_small(const int32_t *prop, int32_t n, int vbits,
                                                            int key_bits, const int32_t *vwgt, int64_t *W,
                                                            int64_t U, const int64_t *capv, int32_t nlabels,
                                                            int32_t *labels, uint8_t *lab8, LPDev *dev) {
    constexpr int NW = kFuseWaves;
    __shared__ uint32_t bufA[kFuseMax], bufB[kFuseMax];
    __shared__ uint32_t wc[NW * 256];  // per (wave, digit) counters, then placement offsets
    __shared__ long long Wl[kFuseLdsLabels];
    __shared__ int32_t tmpi[NW];
    __shared__ uint32_t tmpu[NW];
    __shared__ int32_t wf[NW];
    __shared__ long long wv[NW];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
    const int32_t wbase = w * kFuseWaveSpan;
    const bool wlds = nlabels <= kFuseLdsLabels;
    // everything the round reads from its start state is requested at once
    const int32_t done = dev->done;
    int32_t round = 0, prev_moves = 0;
    if (threadIdx.x == 0) {
        round = dev->round;
        prev_moves = dev->prev_moves;
    }
    int32_t t_of[kFuseRows];
#pragma unroll
    for (int r = 0; r < kFuseRows; r++) {
        const int32_t v = wbase + r * kWave + lane;
        t_of[r] = v < n ? prop[v] : -1;
    }
    if (wlds)
        for (int i = threadIdx.x; i < nlabels; i += kFuseBlock) Wl[i] = W[i];
    // ---- compaction: movers in ascending vertex order
    uint32_t item[kFuseRows];
    int32_t rank[kFuseRows];
    int32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < kFuseRows; r++) {
        const int32_t v = wbase + r * kWave + lane;
        const int32_t t = done ? -1 : t_of[r];
        const uint64_t mb = __ballot(t >= 0);
        item[r] = ((uint32_t)t << vbits) | (uint32_t)v;
        rank[r] = (t >= 0) ? cnt + (int32_t)__popcll(mb & lt) : -1;
        cnt += (int32_t)__popcll(mb);
    }
    int32_t m = 0;
    const int32_t woff = fuse_excl_scan<int32_t>(lane == 0 ? cnt : 0, tmpi, &m);
    const int32_t wstart = __shfl(woff, 0, kWave);
#pragma unroll
    for (int r = 0; r < kFuseRows; r++)
        if (rank[r] >= 0) bufA[wstart + rank[r]] = item[r];
    __syncthreads();
    // ---- stable LSD sort by target, 8 bits a pass
    uint32_t *cur = bufA, *oth = bufB;
    for (int shift = 0; m > 0 && shift < key_bits; shift += 8) {
        const int nb = (key_bits - shift) < 8 ? (key_bits - shift) : 8;
        const uint32_t mask = (1u << nb) - 1u;
        for (int d = threadIdx.x; d < NW * 256; d += kFuseBlock) wc[d] = 0;
        __syncthreads();
        uint32_t dg[kFuseRows];
#pragma unroll
        for (int r = 0; r < kFuseRows; r++) {
            const int32_t p = wbase + r * kWave + lane;
            rank[r] = -1;
            dg[r] = 0;
            if (wbase + r * kWave >= m) continue;  // wave-uniform
            const bool valid = p < m;
            item[r] = valid ? cur[p] : 0u;
            const uint32_t dig = (item[r] >> (vbits + shift)) & mask;
            dg[r] = dig;
            uint64_t peers = __ballot(valid);
            for (int bt = 0; bt < nb; bt++) {
                const bool bit = (dig >> bt) & 1u;
                const uint64_t bm = __ballot(bit);
                peers &= bit ? bm : ~bm;
            }
            const uint32_t before = valid ? wc[w * 256 + dig] : 0u;
            const uint32_t pr = (uint32_t)__popcll(peers & lt);
            if (valid) rank[r] = (int32_t)(before + pr);
            // every lane read the counter before the group's first lane advances it
            if (valid && pr == 0) wc[w * 256 + dig] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // placement offsets in (digit, wave) order: thread i owns digit i / 4, waves 4 (i % 4) .. + 3
        {
            const int d = threadIdx.x >> 2, q0 = (threadIdx.x & 3) * 4;
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                c[j] = wc[(q0 + j) * 256 + d];
                sum += c[j];
            }
            uint32_t tot = 0;
            uint32_t off = fuse_excl_scan<uint32_t>(sum, tmpu, &tot);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                wc[(q0 + j) * 256 + d] = off;
                off += c[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kFuseRows; r++)
            if (rank[r] >= 0) oth[wc[w * 256 + dg[r]] + (uint32_t)rank[r]] = item[r];
        __syncthreads();
        uint32_t *tq = cur;
        cur = oth;
        oth = tq;
    }
    // ---- segmented prefix of mover weights per target, in position order
    const uint32_t vmask = (1u << vbits) - 1u;
    long long pre[kFuseRows];
    bool seen[kFuseRows];
    bool cf = false;  // a segment head at or before the row's end within this wave
    long long cv = 0;
#pragma unroll
    for (int r = 0; r < kFuseRows; r++) {
        const int32_t p = wbase + r * kWave + lane;
        pre[r] = 0;
        seen[r] = false;
        if (wbase + r * kWave >= m) continue;  // wave-uniform
        const bool valid = p < m;
        const uint32_t it = valid ? cur[p] : 0u;
        item[r] = it;
        const long long c = valid ? (long long)vweight(vwgt, (int32_t)(it & vmask)) : 0;
        const bool hd = valid && (p == 0 || (cur[p - 1] >> vbits) != (it >> vbits));
        bool f = hd;
        long long v = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int fo = __shfl_up((int)f, d, kWave);
            const long long vo = __shfl_up(v, d, kWave);
            if (lane >= d) {
                v = f ? v : vo + v;
                f = f || fo;
            }
        }
        if (!f) v += cv;
        f = f || cf;
        pre[r] = v;
        seen[r] = f;
        cf = __shfl(f, kWave - 1, kWave);
        cv = __shfl(v, kWave - 1, kWave);
    }
    if (lane == 0) {
        wf[w] = cf;
        wv[w] = cv;
    }
    __syncthreads();
    long long carry = 0;  // the open segment's sum before this wave
    for (int i = 0; i < w; i++) carry = wf[i] ? wv[i] : carry + wv[i];
    // ---- admission against the weights of the round start
    uint8_t *adm = reinterpret_cast<uint8_t *>(oth);
#pragma unroll
    for (int r = 0; r < kFuseRows; r++) {
        const int32_t p = wbase + r * kWave + lane;
        if (p >= m) continue;
        if (!seen[r]) pre[r] += carry;
        const uint32_t t = item[r] >> vbits;
        const long long wt = wlds ? Wl[t] : W[t];
        adm[p] = (wt + pre[r] <= (capv ? capv[t] : U)) ? 1 : 0;
    }
    __syncthreads();
    // ---- labels and weights
    int32_t moves = 0;
#pragma unroll
    for (int r = 0; r < kFuseRows; r++) {
        const int32_t p = wbase + r * kWave + lane;
        if (p >= m || !adm[p]) continue;
        const uint32_t t = item[r] >> vbits;
        const int32_t vx = (int32_t)(item[r] & vmask);
        const int32_t old = labels[vx];
        const long long c = (long long)vweight(vwgt, vx);
        labels[vx] = (int32_t)t;
        if (lab8) lab8[vx] = (uint8_t)t;
        // admitted movers form a prefix of their target's segment: its last one adds the segment's weight
        const bool tail = p + 1 == m || !adm[p + 1] || (cur[p + 1] >> vbits) != t;
        unsigned long long *wo = wlds ? (unsigned long long *)&Wl[old] : (unsigned long long *)&W[old];
        atomicAdd(wo, (unsigned long long)(-c));
        if (tail) {
            unsigned long long *wt = wlds ? (unsigned long long *)&Wl[t] : (unsigned long long *)&W[t];
            atomicAdd(wt, (unsigned long long)pre[r]);
        }
        moves++;
    }
    int32_t total = 0;
    (void)fuse_excl_scan<int32_t>(moves, tmpi, &total);  // ends with a barrier
    if (wlds)  // this workgroup is the only writer of W in this launch
        for (int i = threadIdx.x; i < nlabels; i += kFuseBlock) W[i] = Wl[i];
    if (threadIdx.x == 0) {  // round bookkeeping (k_round_end with this round's moves)
        dev->round = round + 1;
        if (!done) {
            dev->rounds_run = round + 1;
            dev->total_moves += total;
            if (round >= 1 && total == 0 && prev_moves == 0) dev->done = 1;
            dev->prev_moves = total;
            dev->round_moves = 0;
        }
    }
}

// Few labels: net weight change per label aggregated in LDS first.
__global__ __launch_bounds__(256) void k_apply_w_small(const uint32_t *mk, const int32_t *mv, const int32_t *nmov,
                                                       const int32_t *oldlab, const int32_t *vwgt, int32_t nl,
                                                       int64_t *W) {
    __shared__ unsigned long long h[kSmallLabels];
    const int32_t n = *nmov;
    if ((int64_t)blockIdx.x * blockDim.x >= n) return;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t old = oldlab[p];
        if (old < 0) continue;
        const unsigned long long c = (unsigned long long)vweight(vwgt, mv[p]);
        atomicAdd(&h[mk[p]], c);
        atomicAdd(&h[old], (unsigned long long)(-(long long)c));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nl; i += blockDim.x)
        if (h[i]) atomicAdd((unsigned long long *)&W[i], h[i]);
}

// ---------------------------------------------------------------- active-set rounds
// act[v] = evaluations v still owes (see k_act_step, k_admit, k_act_mark).

__global__ void k_act_fill(uint8_t *act, int32_t n, uint8_t c) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        act[v] = c;
}

// After the proposals: count the edges of the vertices evaluated this round
// and take one owed evaluation off each of them. The others were not in the
// round's lists: their proposal is cleared here.
__global__ __launch_bounds__(256) void k_act_step(const int32_t *xadj, int32_t n, uint8_t *act, int32_t *prop,
                                                  LPDev *dev, int32_t *nbig) {
    __shared__ long long tmp[256 / kWave + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) *nbig = 0;  // the round's list of big movers starts empty
    if (dev->done) return;
    long long vis = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t c = act[v];
        if (c) {
            vis += xadj[v + 1] - xadj[v];
            act[v] = (uint8_t)(c - 1);
        } else {
            prop[v] = -1;
        }
    }
    vis = block_sum<256>(vis, tmp);
    if (threadIdx.x == 0 && vis) atomicAdd((unsigned long long *)&dev->visits, (unsigned long long)vis);
}

// After the admission: every neighbour of an admitted mover owes `renew`
// evaluations. 16 lanes per mover; a mover above kMarkSplit neighbours is
// queued instead as chunks of kMarkChunk entries (list `big`, count `nbig`),
// which k_act_mark_big spreads over whole workgroups.
constexpr int kMarkSplit = 256;
constexpr int kMarkChunk = 4096;
__global__ __launch_bounds__(256) void k_act_mark(const int32_t *mv, const int32_t *oldlab, const int32_t *nmov,
                                                  const int32_t *xadj, const int32_t *adjncy, uint8_t *act,
                                                  uint8_t renew, int2 *big, int32_t *nbig) {
    constexpr int GL = 16;
    const int32_t n = *nmov;
    const int gl = threadIdx.x % GL;
    const int64_t step = (int64_t)gridDim.x * blockDim.x / GL;
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GL; p < n; p += step) {
        if (oldlab[p] < 0) continue;
        const int32_t v = mv[p];
        const int32_t e0 = xadj[v], e1 = xadj[v + 1];
        if (e1 - e0 > kMarkSplit) {
            if (gl == 0) {
                const int32_t nc = (e1 - e0 + kMarkChunk - 1) / kMarkChunk;
                const int32_t at = atomicAdd(nbig, nc);
                for (int32_t q = 0; q < nc; q++) big[at + q] = make_int2(v, e0 + q * kMarkChunk);
            }
            continue;
        }
        for (int32_t e = e0 + gl; e < e1; e += GL) act[adjncy[e]] = renew;
    }
}

__global__ __launch_bounds__(256) void k_act_mark_big(const int2 *big, const int32_t *nbig, const int32_t *xadj,
                                                      const int32_t *adjncy, uint8_t *act, uint8_t renew) {
    const int32_t nb = *nbig;
    for (int64_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const int2 c = big[i];
        const int32_t e1 = min(xadj[c.x + 1], c.y + kMarkChunk);
        for (int32_t e = c.y + threadIdx.x; e < e1; e += 256) act[adjncy[e]] = renew;
    }
}

// Active-set rounds: each round's tier lists keep the vertices that owe an
// evaluation (compaction in tier order, then the tier starts by binary search).
struct TierStarts {
    int64_t s[kTiers + 1];
};
__global__ void k_set_starts(TierStarts h, int64_t *ts) {
    if (threadIdx.x <= kTiers) ts[threadIdx.x] = h.s[threadIdx.x];
}
struct ActFlag {
    const int32_t *verts;
    const uint8_t *act;
    const int32_t *done;
    __device__ bool operator()(int64_t i) const { return !*done && act[verts[i]] > 0; }
};
struct ActEmit {
    const int32_t *verts;  // full tier-ordered list
    int32_t *averts;
    uint8_t *atier;
    TierStarts ts;
    int64_t first;  // list entries before `first` (tier 0) are not scanned
    __device__ void operator()(int64_t i, int32_t pos) const {
        const int64_t j = first + i;
        averts[pos] = verts[j];
        int t = 1;
        while (t < kTiers - 1 && j >= ts.s[t + 1]) t++;
        atier[pos] = (uint8_t)t;
    }
};
__global__ void k_act_bounds(const uint8_t *atier, const int32_t *count, int64_t *ts) {
    const int t = threadIdx.x;
    if (t > kTiers) return;
    const int32_t c = *count;
    if (t == kTiers) {
        ts[t] = c;
        return;
    }
    int32_t lo = 0, hi = c;  // first position whose tier is >= t
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int)atier[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    ts[t] = lo;
}

__global__ void k_round_end_groups(GroupState *gs, int32_t ng) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < ng; q += gridDim.x * blockDim.x) {
        GroupState st = gs[q];
        const int32_t r = st.seen;
        st.seen = r + 1;
        if (!st.done) {
            st.rounds_run = r + 1;
            st.total += st.moves;
            if (r >= 1 && st.moves == 0 && st.prev == 0) st.done = 1;
            st.prev = st.moves;
        }
        st.moves = 0;
        gs[q] = st;
    }
}

__global__ void k_round_end(LPDev *dev) {
    const int32_t r = dev->round;
    dev->round = r + 1;
    if (dev->done) return;
    const int32_t m = dev->round_moves;
    dev->rounds_run = r + 1;
    dev->total_moves += m;
    if (r >= 1 && m == 0 && dev->prev_moves == 0) dev->done = 1;
    dev->prev_moves = m;
    dev->round_moves = 0;
}

__global__ void k_label_weights(const int32_t *labels, const int32_t *vwgt, int32_t n, int64_t *W) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t L = labels[v];
        if (L >= 0) atomicAdd((unsigned long long *)&W[L], (unsigned long long)vweight(vwgt, (int32_t)v));
    }
}

// Many vertices per label but too many labels for one LDS array (the blocks of
// a batch of graphs): a workgroup sums a span of consecutive vertices in an
// LDS hash keyed by label, a wave on one label inserting once, and adds each
// slot to W at the end; a label that finds no slot in 8 probes goes to W
// directly.
constexpr int kLwLog = 11;
constexpr int kLwSlots = 1 << kLwLog;
constexpr int kLwSpan = 16384;
__global__ __launch_bounds__(256) void k_label_weights_hash(const int32_t *labels, const int32_t *vwgt, int32_t n,
                                                            int64_t *W) {
    __shared__ int32_t key[kLwSlots];
    __shared__ unsigned long long val[kLwSlots];
    const int lane = lane_id();
    for (int64_t base = (int64_t)blockIdx.x * kLwSpan; base < n; base += (int64_t)gridDim.x * kLwSpan) {
        for (int i = threadIdx.x; i < kLwSlots; i += blockDim.x) {
            key[i] = -1;
            val[i] = 0;
        }
        __syncthreads();
        const int64_t end = min(base + kLwSpan, (int64_t)n);
        for (int64_t v = base + threadIdx.x; v - lane < end; v += blockDim.x) {
            const bool valid = v < end;
            const int32_t L = valid ? labels[v] : -1;
            bool todo = L >= 0;
            const uint64_t vm = __ballot(todo);
            if (!vm) continue;
            unsigned long long x = todo ? (unsigned long long)vweight(vwgt, (int32_t)v) : 0ull;
            int32_t Lx = L;
            const int32_t L0 = __shfl(L, __ffsll((unsigned long long)vm) - 1, kWave);
            if (__ballot(todo && L != L0) == 0) {
                x = wave_sum(x);
                todo = lane == 0;
                Lx = L0;
            }
            if (!todo) continue;
            uint32_t h = ((uint32_t)Lx * 2654435761u) >> (32 - kLwLog);
            bool placed = false;
            for (int probe = 0; probe < 8 && !placed; probe++) {
                const int32_t k = atomicCAS(&key[h], -1, Lx);
                if (k == -1 || k == Lx) {
                    atomicAdd(&val[h], x);
                    placed = true;
                } else {
                    h = (h + 1) & (kLwSlots - 1);
                }
            }
            if (!placed) atomicAdd((unsigned long long *)&W[Lx], x);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kLwSlots; i += blockDim.x)
            if (key[i] >= 0 && val[i]) atomicAdd((unsigned long long *)&W[key[i]], val[i]);
        __syncthreads();
    }
}

// Few labels (k-way partitions): per-block LDS totals, then one global atomic per label and block.
__global__ __launch_bounds__(256) void k_label_weights_small(const int32_t *labels, const int32_t *vwgt, int32_t n,
                                                             int32_t nl, int64_t *W) {
    __shared__ unsigned long long h[kSmallLabels];
    for (int i = threadIdx.x; i < nl; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t L = labels[v];
        if (L >= 0) atomicAdd(&h[L], (unsigned long long)vweight(vwgt, (int32_t)v));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nl; i += blockDim.x)
        if (h[i]) atomicAdd((unsigned long long *)&W[i], h[i]);
}

struct EdgeWeightIn {
    const int32_t *w;
    __device__ int64_t operator()(int64_t i) const { return (int64_t)w[i]; }
};
struct NoOut64 {
    __device__ void operator()(int64_t, int64_t, int64_t) const {}
};

template <typename AccT>
int launch_proposals(const LPArgs &a, const int32_t *verts, const int64_t *tstart, TierList tl,
                     const int32_t *hub_log, const int64_t *hub_off, int32_t *gkey, AccT *gval, hipStream_t s,
                     const double *tb, bool skip_hubs) {
    const char *acc = sizeof(AccT) == 4 ? "int" : "long";
    auto cnt = [&](int t) { return (int32_t)(tstart[t + 1] - tstart[t]); };
    auto lst = [&](int t) { return verts + tstart[t]; };
    constexpr int NW = kPropBlock / kWave;
    // blocks: enough waves to cover the tier, capped so each block loops a few times
    auto blocks_for = [&](int32_t c, int per_block) { return grid_for(c, per_block, 16384); };
    int32_t c;
    if ((c = cnt(1)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH("k_plane<4, int>", tb[1], s, hipLaunchKernelGGL((k_plane<4, 4>), dim3(blocks_for(c, NW * 16)), dim3(kPropBlock), 0, s,
                           a, tl, 1)); else GP_PROF_LAUNCH((std::string("k_propose_group<4, 8, ") + acc + ">").c_str(), tb[1], s, hipLaunchKernelGGL((k_propose_group<4, 8, AccT>), dim3(blocks_for(c, NW * 16)), dim3(kPropBlock), 0, s,
                           a, tl, 1));
    }
    if ((c = cnt(2)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH("k_plane<8, int>", tb[2], s, hipLaunchKernelGGL((k_plane<8, 8>), dim3(blocks_for(c, NW * 8)), dim3(kPropBlock), 0, s,
                           a, tl, 2)); else GP_PROF_LAUNCH((std::string("k_propose_group<8, 16, ") + acc + ">").c_str(), tb[2], s, hipLaunchKernelGGL((k_propose_group<8, 16, AccT>), dim3(blocks_for(c, NW * 8)), dim3(kPropBlock), 0, s,
                           a, tl, 2));
    }
    if ((c = cnt(3)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH((std::string("k_pgroup<16, 32, ") + acc + ">").c_str(), tb[3], s, hipLaunchKernelGGL((k_pgroup<16, 32>), dim3(blocks_for(c, NW * 4)), dim3(kPropBlock), 0,
                           s, a, tl, 3)); else GP_PROF_LAUNCH((std::string("k_propose_group<16, 32, ") + acc + ">").c_str(), tb[3], s, hipLaunchKernelGGL((k_propose_group<16, 32, AccT>), dim3(blocks_for(c, NW * 4)), dim3(kPropBlock), 0,
                           s, a, tl, 3));
    }
    if ((c = cnt(4)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH((std::string("k_pgroup<32, 128, ") + acc + ">").c_str(), tb[4], s, hipLaunchKernelGGL((k_pgroup<32, 128>), dim3(blocks_for(c, NW * 2)), dim3(kPropBlock), 0,
                           s, a, tl, 4)); else GP_PROF_LAUNCH((std::string("k_propose_group<32, 128, ") + acc + ">").c_str(), tb[4], s, hipLaunchKernelGGL((k_propose_group<32, 128, AccT>), dim3(blocks_for(c, NW * 2)), dim3(kPropBlock), 0,
                           s, a, tl, 4));
    }
    if ((c = cnt(5)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH((std::string("k_pgroup<64, 512, ") + acc + ">").c_str(), tb[5], s, hipLaunchKernelGGL((k_pgroup<64, 512>), dim3(blocks_for(c, NW)), dim3(kPropBlock), 0, s,
                           a, tl, 5)); else GP_PROF_LAUNCH((std::string("k_propose_group<64, 512, ") + acc + ">").c_str(), tb[5], s, hipLaunchKernelGGL((k_propose_group<64, 512, AccT>), dim3(blocks_for(c, NW)), dim3(kPropBlock), 0, s,
                           a, tl, 5));
    }
    if ((c = cnt(6)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH((std::string("k_pblock<128, 2048, ") + acc + ">").c_str(), tb[6], s, hipLaunchKernelGGL((k_pblock<128, 2048>), dim3(grid_for(c, 1, 16384)), dim3(128), 0, s, a,
                           tl, 6)); else GP_PROF_LAUNCH((std::string("k_propose_block<128, 2048, ") + acc + ">").c_str(), tb[6], s, hipLaunchKernelGGL((k_propose_block<128, 2048, AccT>), dim3(grid_for(c, 1, 16384)), dim3(128), 0, s, a,
                           tl, 6));
    }
    if ((c = cnt(7)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH((std::string("k_pblock<256, 4096, ") + acc + ">").c_str(), tb[7], s, hipLaunchKernelGGL((k_pblock<256, 4096>), dim3(grid_for(c, 1, 8192)), dim3(256), 0, s, a,
                           tl, 7)); else GP_PROF_LAUNCH((std::string("k_propose_block<256, 4096, ") + acc + ">").c_str(), tb[7], s, hipLaunchKernelGGL((k_propose_block<256, 4096, AccT>), dim3(grid_for(c, 1, 8192)), dim3(256), 0, s, a,
                           tl, 7));
    }
    if ((c = cnt(8)) > 0) {
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH("k_pblock<512, 8192, int>", tb[8], s, hipLaunchKernelGGL((k_pblock<512, 8192>), dim3(grid_for(c, 1, 4096)), dim3(512), 0, s, a, tl, 8));
        else GP_PROF_LAUNCH((std::string("k_propose_block<1024, 8192, ") + acc + ">").c_str(), tb[8], s, hipLaunchKernelGGL((k_propose_block<1024, 8192, AccT>), dim3(grid_for(c, 1, 2048)), dim3(1024), 0, s, a,
                           tl, 8));
    }
    if ((c = cnt(9)) > 0) {  // 64-bit sums: the tier is empty (its cap is tier 8's)
        if constexpr (sizeof(AccT) == 4) GP_PROF_LAUNCH("k_pblock<1024, 16384, int>", tb[9], s, hipLaunchKernelGGL((k_pblock<1024, 16384>), dim3(grid_for(c, 1, 2048)), dim3(1024), 0, s, a, tl, 9));
        else GP_PROF_LAUNCH((std::string("k_propose_block<1024, 8192, ") + acc + ">").c_str(), tb[9], s, hipLaunchKernelGGL((k_propose_block<1024, 8192, AccT>), dim3(grid_for(c, 1, 2048)), dim3(1024), 0, s, a,
                           tl, 9));
    }
    constexpr int H = kTiers - 1;
    if (!skip_hubs && (c = cnt(H)) > 0) {
        GP_PROF_LAUNCH((std::string("k_propose_hub<1024, ") + acc + ">").c_str(), tb[H], s, hipLaunchKernelGGL((k_propose_hub<1024, AccT>), dim3(c), dim3(1024), 0, s, a, lst(H), c, hub_off,
                           hub_log, gkey, gval));
    }
    GP_LAUNCH_CHECK();
    return GP_OK;
}

// GP_ROUND_GRAPHS=1 records one round's launch sequence once per LP run and
// replays it as a HIP graph for the later rounds; unset or 0, every round is
// launched directly (faster on this stack: a graph launch costs the host more
// than the few launches of a round it replaces). Read at every LP run.
bool use_round_graphs() {
    const char *e = std::getenv("GP_ROUND_GRAPHS");
    return e && e[0] == '1';
}

// A library-owned stream (default priority) used only to record launch
// sequences; recorded graphs are launched on the caller's stream.
hipStream_t capture_stream() {
    static thread_local hipStream_t cs = nullptr;
    if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) cs = nullptr;
    return cs;
}

}  // namespace

Tuning &tuning() {
    static Tuning t;
    return t;
}

int set_tuning(const Tuning &t) {
    const int32_t *b = t.tier_max;
    const bool ok = b[0] >= tier_cap(3, false) && b[0] <= tier_cap(4, false) && b[1] >= b[0] &&
                    b[1] <= tier_cap(5, false) && b[2] >= b[1] && b[2] <= tier_cap(7, false) && b[3] >= b[2] &&
                    b[3] <= tier_cap(9, false) && t.dense_split >= 16 && t.dense_split <= (1 << 30) &&
                    t.dense_chunk >= 256 && t.dense_chunk <= 65536 && t.dense_chunk % 256 == 0;
    if (!ok) {
        set_error("tuning: tier bounds must be non-decreasing within 16..64, ..256, ..2048, ..8192; dense_split in "
                  "16..2^30; dense_chunk a multiple of 256 in 256..65536");
        return GP_ERR_ARG;
    }
    tuning() = t;
    return GP_OK;
}

// Upper bound of the scratch one lp_run holds at once (the allocations of
// lp_run below, each rounded up to 256 bytes, with every per-vertex count
// taken at n and every per-entry count at nnz), under the current tuning.
// Scan, compaction and sort temporaries are reusable slots that grow by
// 1.25x at a time and keep their outgrown buffers until the run ends: at most
// 1.25 / (1 - 1/1.25) = 6.25 times their final size, i.e. 6.25 * n / 4 bytes
// of radix histograms, 6.25 * 2 * 8 * ceil(m / 2048) bytes per scan depth,
// plus 256 bytes of rounding per growth.
size_t lp_scratch_bound(int64_t n, int64_t nnz, int64_t nlabels, bool active) {
    auto R = [](double x) { return (double)((((size_t)std::ceil(x > 1 ? x : 1)) + 255) & ~(size_t)255); };
    const Tuning &tu = tuning();
    const bool dense = nlabels <= kDenseLabels;
    double worst = 0;
    for (int wi = 0; wi < 2; wi++) {
        const bool wide = wi == 1;
        double b = 0;
        b += 4 * R(4.0 * n) + R(40) + R(80) + R(8 * (kTiers + 1));  // tier keys and values, counts, starts
        if (active) b += R(4.0 * n) + R(n) + R(4) + R(8 * (kTiers + 1));
        const int32_t b4 = std::min(tu.tier_max[0], tier_cap(4, wide));
        const int32_t b5 = std::max(std::min(tu.tier_max[1], tier_cap(5, wide)), b4);
        const int32_t b6 = std::max(std::min(tu.tier_max[2], tier_cap(6, wide)), b5);
        const int32_t b7 = std::max(std::min(tu.tier_max[2], tier_cap(7, wide)), b6);
        const int32_t bh = std::max(std::min(tu.tier_max[3], tier_cap(9, wide)), b7);
        if (!dense) {
            const double nh = (double)std::min<int64_t>(n, nnz / ((int64_t)bh + 1));
            const double ttot = 4.0 * nnz;
            if (!wide) {
                const double nchunks = (double)nnz / kHubChunk + nh, nslices = ttot / kHubSlice + nh,
                             nbuckets = (double)nnz / kHubPer + nh;
                b += 8 * R(4 * nh) + 4 * R(8 * nh) + R(12) + R(8);
                b += R(4 * nchunks) + R(4 * nslices) + 2 * R(4 * nbuckets) + 2 * R(4 * ttot) +
                     R(8.0 * nbuckets * kBucketCap);
            } else {
                b += R(4 * nh) + 2 * R(8 * nh) + R(8) + R(4 * ttot) + R(8 * ttot);
            }
        } else {
            const int32_t split = std::max(b4, tu.dense_split);
            const double nbig = (double)std::min<int64_t>(n, nnz / ((int64_t)split + 1));
            const double dchunks = (double)nnz / tu.dense_chunk + nbig;
            const int KT = nlabels <= 16 ? 16 : (nlabels <= 64 ? 64 : 256);
            b += 2 * R(4 * nbig) + R(4) + R(8 * nbig) + R(16 * dchunks) + R(nbig * KT * (wide ? 8.0 : 4.0));
            b += R(n);  // byte labels
        }
        b += 6 * R(4.0 * n) + R(4) + R(4.0 * nlabels) + R(8.0 * n) + R(sizeof(LPDev));  // per-round buffers
        if (active) b += R(n) + R(8.0 * ((double)nnz / kMarkChunk + (double)nnz / kMarkSplit + 1)) + R(4);
        worst = std::max(worst, b);
    }
    const double m = (double)std::max<int64_t>(n, 1);
    const double temps = 6.25 * (m / 4.0) + 6.25 * 2 * 8 * 4 * std::ceil(m / kScanTile) + 128.0 * 1024;
    return (size_t)(worst + temps);
}

int total_edge_weight(const DevGraph &g, int64_t *out, Scratch &sc) {
    if (!g.adjwgt) {
        *out = g.nnz;
        return GP_OK;
    }
    int64_t *d = nullptr;
    GP_TRY(sc.alloc(&d, 1));
    GP_TRY((scan<int64_t>(EdgeWeightIn{g.adjwgt}, NoOut64{}, g.nnz, nullptr, d, sc)));
    GP_HIP(hipMemcpyAsync(out, d, sizeof(int64_t), hipMemcpyDeviceToHost, sc.stream()));
    GP_HIP(hipStreamSynchronize(sc.stream()));
    return GP_OK;
}

int label_weights(const DevGraph &g, const int32_t *labels, int64_t *W, int32_t nlabels, Scratch &sc) {
    GP_HIP(hipMemsetAsync(W, 0, sizeof(int64_t) * (size_t)(nlabels > 0 ? nlabels : 1), sc.stream()));
    if (g.n > 0) {
        if (nlabels <= kSmallLabels)
            hipLaunchKernelGGL(k_label_weights_small, dim3(grid_for(g.n, 256, 1024)), dim3(256), 0, sc.stream(),
                               labels, g.vwgt, g.n, nlabels, W);
        else if ((int64_t)nlabels * 4 <= g.n)
            hipLaunchKernelGGL(k_label_weights_hash, dim3(grid_for(g.n, kLwSpan, 4096)), dim3(256), 0, sc.stream(),
                               labels, g.vwgt, g.n, W);
        else
            hipLaunchKernelGGL(k_label_weights, dim3(grid_for(g.n, 256, 65536)), dim3(256), 0, sc.stream(), labels,
                               g.vwgt, g.n, W);
        GP_LAUNCH_CHECK();
    }
    return GP_OK;
}

int lp_run(const DevGraph &g, int32_t *labels, int64_t *W, int32_t nlabels, int64_t U, int32_t rounds,
           int32_t dir_alternate, bool wide, LPOut *out, Scratch &sc, const int64_t *capv, const uint8_t *frozen,
           const int32_t *group, int32_t ngroups, bool active) {
    // everything below is internal to the call (results are written in place
    // or read back to the host): its scratch is given back on every return
    ScratchScope scope(sc);
    hipStream_t s = sc.stream();
    const int32_t n = g.n;
    if (n == 0 || rounds == 0) {
        if (out) *out = LPOut{};
        return GP_OK;
    }
    // ---- degree tiers (once per call)
    uint32_t *tkey = nullptr, *tkey2 = nullptr;
    int32_t *tval = nullptr, *tval2 = nullptr, *tcnt = nullptr;
    GP_TRY(sc.alloc(&tkey, n));
    GP_TRY(sc.alloc(&tkey2, n));
    GP_TRY(sc.alloc(&tval, n));
    GP_TRY(sc.alloc(&tval2, n));
    unsigned long long *tedge = nullptr;
    GP_TRY(sc.alloc(&tcnt, kTiers));
    GP_TRY(sc.alloc(&tedge, kTiers));
    GP_HIP(hipMemsetAsync(tcnt, 0, sizeof(int32_t) * kTiers, s));
    GP_HIP(hipMemsetAsync(tedge, 0, sizeof(unsigned long long) * kTiers, s));
    TierKey tk{g.xadj, labels, frozen, wide, {}};
    {
        const Tuning &tu = tuning();
        const bool dense_tiers = nlabels <= kDenseLabels;
        for (int t = 0; t < kTiers; t++) tk.bound[t] = tier_cap(t, wide);
        // tuned bounds: 32 lanes, 64 lanes, workgroups (split at 1024 between
        // the 128- and 256-thread kernels), 1024-thread workgroups
        tk.bound[4] = std::min(tu.tier_max[0], tier_cap(4, wide));
        tk.bound[5] = std::min(tu.tier_max[1], tier_cap(5, wide));
        tk.bound[6] = std::min(tu.tier_max[2], tier_cap(6, wide));
        tk.bound[7] = std::min(tu.tier_max[2], tier_cap(7, wide));
        tk.bound[8] = std::min(tu.tier_max[3], tier_cap(8, wide));
        tk.bound[9] = std::min(tu.tier_max[3], tier_cap(9, wide));
        if (dense_tiers) {  // dense tables have no degree limit: rows above the split are chunked
            tk.bound[5] = std::max(tk.bound[4], tu.dense_split);
            tk.bound[6] = tk.bound[7] = tk.bound[8] = tk.bound[9] = tk.bound[5];
        }
        for (int t = 1; t < kTiers - 1; t++) tk.bound[t] = std::max(tk.bound[t], tk.bound[t - 1]);
    }
    hipLaunchKernelGGL(k_tier_keys, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, tk, n, tkey, tval, tcnt, tedge);
    GP_LAUNCH_CHECK();
    GP_TRY((radix_sort<uint32_t, int32_t>(&tkey, &tval, &tkey2, &tval2, n, nullptr, 4, sc)));
    int32_t hcnt[kTiers];
    unsigned long long hedge[kTiers];
    GP_HIP(hipMemcpyAsync(hcnt, tcnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(hedge, tedge, sizeof(hedge), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    int64_t tstart[kTiers + 1];
    tstart[0] = 0;
    for (int t = 0; t < kTiers; t++) tstart[t + 1] = tstart[t] + hcnt[t];
    const int32_t *verts = tval;
    const bool dense_mode = nlabels <= kDenseLabels;
    // Algorithmic bytes of one proposal pass over tier t: per edge the
    // neighbour id, its weight (when present) and its label (one byte with
    // dense tables); per vertex the
    // tier-list entry, the two row offsets, the own label, the proposal
    // write, the vertex weight (when present) and, for hashed tables, the
    // weight of the chosen label.
    const double per_edge = 4.0 + (g.adjwgt ? 4.0 : 0.0) + (dense_mode ? 1.0 : 4.0);
    const double per_vertex = 4.0 + 8.0 + 4.0 + 4.0 + (g.vwgt ? 4.0 : 0.0) + (dense_mode ? 0.0 : 8.0);
    double tbytes[kTiers + 1];
    for (int t = 0; t < kTiers; t++) tbytes[t] = (double)hedge[t] * per_edge + (double)hcnt[t] * per_vertex;
    tbytes[kTiers] = 0;

    // the tier starts on the device; in active-set rounds the kernels read
    // per-round lists of the vertices that owe an evaluation instead
    int64_t *ts_dev = nullptr;
    GP_TRY(sc.alloc(&ts_dev, kTiers + 1));
    TierStarts tsh;
    for (int t = 0; t <= kTiers; t++) tsh.s[t] = tstart[t];
    hipLaunchKernelGGL(k_set_starts, dim3(1), dim3(64), 0, s, tsh, ts_dev);
    GP_LAUNCH_CHECK();
    TierList tl{verts, ts_dev};
    int32_t *averts = nullptr, *acount = nullptr;
    uint8_t *atier = nullptr;
    int64_t *ats = nullptr;
    const int64_t afirst = tstart[1];
    if (active) {
        GP_TRY(sc.alloc(&averts, n));
        GP_TRY(sc.alloc(&atier, n));
        GP_TRY(sc.alloc(&acount, 1));
        GP_TRY(sc.alloc(&ats, kTiers + 1));
        GP_HIP(hipMemsetAsync(ats, 0, sizeof(int64_t) * (kTiers + 1), s));
        tl = TierList{averts, ats};
    }

    // ---- hub tables (hashed tables only; dense tables need none)
    const bool dense = nlabels <= kDenseLabels;
    const int32_t nh = dense ? 0 : hcnt[kTiers - 1];
    const bool split_hubs = nh > 0 && !wide;
    int32_t *hub_log = nullptr, *gkey = nullptr;
    int64_t *hub_off = nullptr;
    void *gval = nullptr;
    HubPlan hp{};
    int32_t nchunks = 0, nslices = 0, nbuckets = 0;
    if (split_hubs) {
        const int32_t *hubs = verts + tstart[kTiers - 1];
        int32_t *tlog = nullptr, *nch = nullptr, *nsl = nullptr, *nbk = nullptr, *cfirst = nullptr,
                *sfirst = nullptr, *bfirst = nullptr, *d_tot = nullptr, *chub = nullptr, *shub = nullptr,
                *bhub = nullptr, *fill = nullptr, *ovf = nullptr;
        int64_t *tcap = nullptr, *toff = nullptr, *d_ttot = nullptr;
        unsigned long long *own = nullptr, *best = nullptr;
        GP_TRY(sc.alloc(&tlog, nh));
        GP_TRY(sc.alloc(&nch, nh));
        GP_TRY(sc.alloc(&nsl, nh));
        GP_TRY(sc.alloc(&nbk, nh));
        GP_TRY(sc.alloc(&cfirst, nh));
        GP_TRY(sc.alloc(&sfirst, nh));
        GP_TRY(sc.alloc(&bfirst, nh));
        GP_TRY(sc.alloc(&d_tot, 3));
        GP_TRY(sc.alloc(&tcap, nh));
        GP_TRY(sc.alloc(&toff, nh));
        GP_TRY(sc.alloc(&d_ttot, 1));
        GP_TRY(sc.alloc(&own, nh));
        GP_TRY(sc.alloc(&best, nh));
        GP_TRY(sc.alloc(&ovf, nh));
        hipLaunchKernelGGL(k_hub_plan, dim3(grid_for(nh, 256, 1024)), dim3(256), 0, s, g.xadj, hubs, nh, tlog, tcap,
                           nch, nsl, nbk);
        GP_LAUNCH_CHECK();
        GP_TRY((scan<int64_t>(LoadIn<int64_t>{tcap}, StoreExcl<int64_t>{toff}, nh, nullptr, d_ttot, sc)));
        GP_TRY((scan<int32_t>(LoadIn<int32_t>{nch}, StoreExcl<int32_t>{cfirst}, nh, nullptr, d_tot, sc)));
        GP_TRY((scan<int32_t>(LoadIn<int32_t>{nsl}, StoreExcl<int32_t>{sfirst}, nh, nullptr, d_tot + 1, sc)));
        GP_TRY((scan<int32_t>(LoadIn<int32_t>{nbk}, StoreExcl<int32_t>{bfirst}, nh, nullptr, d_tot + 2, sc)));
        int32_t tots[3];
        int64_t ttot = 0;
        GP_HIP(hipMemcpyAsync(tots, d_tot, sizeof(tots), hipMemcpyDeviceToHost, s));
        GP_HIP(hipMemcpyAsync(&ttot, d_ttot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        nchunks = tots[0];
        nslices = tots[1];
        nbuckets = tots[2];
        GP_TRY(sc.alloc(&chub, nchunks));
        GP_TRY(sc.alloc(&shub, nslices));
        GP_TRY(sc.alloc(&bhub, nbuckets));
        GP_TRY(sc.alloc(&fill, nbuckets));
        hipLaunchKernelGGL(k_hub_expand, dim3(grid_for(nh, 256, 1024)), dim3(256), 0, s, cfirst, nch, nh, chub);
        hipLaunchKernelGGL(k_hub_expand, dim3(grid_for(nh, 256, 1024)), dim3(256), 0, s, sfirst, nsl, nh, shub);
        hipLaunchKernelGGL(k_hub_expand, dim3(grid_for(nh, 256, 1024)), dim3(256), 0, s, bfirst, nbk, nh, bhub);
        GP_LAUNCH_CHECK();
        int32_t *tk = nullptr, *tv = nullptr;
        int2 *pairs = nullptr;
        GP_TRY(sc.alloc(&tk, ttot));
        GP_TRY(sc.alloc(&tv, ttot));
        GP_TRY(sc.alloc(&pairs, (int64_t)nbuckets * kBucketCap));
        GP_HIP(hipMemsetAsync(tk, 0xFF, sizeof(int32_t) * (size_t)ttot, s));
        GP_HIP(hipMemsetAsync(tv, 0, sizeof(int32_t) * (size_t)ttot, s));
        GP_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * nbuckets, s));
        GP_HIP(hipMemsetAsync(own, 0, sizeof(unsigned long long) * nh, s));
        GP_HIP(hipMemsetAsync(best, 0, sizeof(unsigned long long) * nh, s));
        GP_HIP(hipMemsetAsync(ovf, 0, sizeof(int32_t) * nh, s));
        hp = HubPlan{hubs, toff, tlog, chub, cfirst, shub, sfirst, nbk, bfirst, bhub, fill, pairs, tk, tv, ovf, own,
                     best};
    } else if (nh > 0) {
        int64_t *hcap = nullptr, *htot = nullptr;
        GP_TRY(sc.alloc(&hub_log, nh));
        GP_TRY(sc.alloc(&hcap, nh));
        GP_TRY(sc.alloc(&hub_off, nh));
        GP_TRY(sc.alloc(&htot, 1));
        hipLaunchKernelGGL(k_hub_caps, dim3(grid_for(nh, 256, 1024)), dim3(256), 0, s, g.xadj,
                           verts + tstart[kTiers - 1], nh, hub_log, hcap);
        GP_LAUNCH_CHECK();
        GP_TRY((scan<int64_t>(LoadIn<int64_t>{hcap}, StoreExcl<int64_t>{hub_off}, nh, nullptr, htot, sc)));
        int64_t total = 0;
        GP_HIP(hipMemcpyAsync(&total, htot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        GP_TRY(sc.alloc(&gkey, total));
        GP_HIP(hipMemsetAsync(gkey, 0xFF, sizeof(int32_t) * (size_t)total, s));
        int64_t *p = nullptr;
        GP_TRY(sc.alloc(&p, total));
        GP_HIP(hipMemsetAsync(p, 0, sizeof(int64_t) * (size_t)total, s));
        gval = p;
    }

    // ---- dense mode: chunk plan for vertices above the group tiers
    DenseBig db{};
    int32_t dchunks = 0;
    const int32_t nbig = dense ? (int32_t)(tstart[kTiers] - tstart[6]) : 0;
    if (nbig > 0) {
        const int KT = nlabels <= 16 ? 16 : (nlabels <= 64 ? 64 : 256);
        const int32_t *big = verts + tstart[6];
        int32_t *num = nullptr, *first = nullptr, *d_tot = nullptr;
        int4 *desc = nullptr;
        unsigned long long *own = nullptr;
        GP_TRY(sc.alloc(&num, nbig));
        GP_TRY(sc.alloc(&first, nbig));
        GP_TRY(sc.alloc(&d_tot, 1));
        GP_TRY(sc.alloc(&own, nbig));
        const int32_t chunk = tuning().dense_chunk;
        hipLaunchKernelGGL(k_chunk_counts, dim3(grid_for(nbig, 256, 4096)), dim3(256), 0, s, g.xadj, big, nbig,
                           chunk, num);
        GP_LAUNCH_CHECK();
        GP_TRY((scan<int32_t>(LoadIn<int32_t>{num}, StoreExcl<int32_t>{first}, nbig, nullptr, d_tot, sc)));
        GP_HIP(hipMemcpyAsync(&dchunks, d_tot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        GP_TRY(sc.alloc(&desc, dchunks));
        hipLaunchKernelGGL(k_chunk_desc, dim3(grid_for(nbig, 256, 4096)), dim3(256), 0, s, g.xadj, big, first, num,
                           nbig, chunk, desc);
        GP_LAUNCH_CHECK();
        const size_t cb = (size_t)nbig * KT * (wide ? sizeof(int64_t) : sizeof(int32_t));
        void *gconn = nullptr;
        GP_TRY(sc.alloc((char **)&gconn, cb));
        GP_HIP(hipMemsetAsync(gconn, 0, cb, s));
        GP_HIP(hipMemsetAsync(own, 0, sizeof(unsigned long long) * nbig, s));
        db = DenseBig{big, desc, gconn, own, nbig, chunk};
    }

    // ---- dense mode: byte copy of the labels (block ids < 256) for the
    // neighbour gathers, a quarter of the int32 footprint in L2; labels that
    // take no part (-1) belong to vertices without neighbours, never gathered
    uint8_t *lab8 = nullptr;
    if (dense) {
        GP_TRY(sc.alloc(&lab8, n));
        hipLaunchKernelGGL(k_labels_u8, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, labels, n, lab8);
        GP_LAUNCH_CHECK();
    }

    // ---- per-round buffers
    int32_t *prop = nullptr, *mv = nullptr, *mv2 = nullptr, *nmov = nullptr, *headpos = nullptr,
            *oldlab = nullptr;
    uint32_t *mk = nullptr, *mk2 = nullptr;
    int64_t *S = nullptr;
    LPDev *dev = nullptr;
    GP_TRY(sc.alloc(&prop, n));
    GP_TRY(sc.alloc(&mk, n));
    GP_TRY(sc.alloc(&mk2, n));
    GP_TRY(sc.alloc(&mv, n));
    GP_TRY(sc.alloc(&mv2, n));
    GP_TRY(sc.alloc(&nmov, 1));
    GP_TRY(sc.alloc(&headpos, nlabels));
    GP_TRY(sc.alloc(&oldlab, n));
    GP_TRY(sc.alloc(&S, n));
    GP_TRY(sc.alloc(&dev, 1));
    GP_HIP(hipMemsetAsync(prop, 0xFF, sizeof(int32_t) * (size_t)n, s));
    GP_HIP(hipMemsetAsync(dev, 0, sizeof(LPDev), s));
    GroupState *gstate = nullptr;
    if (group && ngroups > 0) {
        GP_TRY(sc.alloc(&gstate, ngroups));
        GP_HIP(hipMemsetAsync(gstate, 0, sizeof(GroupState) * (size_t)ngroups, s));
    } else {
        group = nullptr;
    }
    const int key_bits = bits_for(nlabels > 0 ? nlabels - 1 : 0);
    const int vbits = bits_for(n > 0 ? n - 1 : 0);
    const bool fuse_rest = !group && !active && n <= kFuseMax && vbits + key_bits <= 32;
    // active-set rounds: every vertex starts owing one evaluation per direction
    const uint8_t renew = dir_alternate ? 2 : 1;
    uint8_t *act = nullptr;
    int2 *mbig = nullptr;
    int32_t *nmbig = nullptr;
    if (active) {
        GP_TRY(sc.alloc(&act, n));
        // chunks of the movers above kMarkSplit neighbours: at most
        // nnz / kMarkChunk + nnz / kMarkSplit of them
        GP_TRY(sc.alloc(&mbig, (size_t)g.nnz / kMarkChunk + (size_t)g.nnz / kMarkSplit + 1));
        GP_TRY(sc.alloc(&nmbig, 1));
        GP_HIP(hipMemsetAsync(nmbig, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_act_fill, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, act, n, renew);
        GP_LAUNCH_CHECK();
    }

    // ---- dense mode: connection rows of the vertices above KT/8 neighbours
    // (the plain rounds keep gathering for the others). Not for the levels
    // whose round tail runs in one workgroup, nor in a caller's workspace or
    // the static scratch, whose bounds are those of the plain rounds.
    RowTables rt;
    const int KTd = nlabels <= 16 ? 16 : (nlabels <= 64 ? 64 : 256);
    if (dense && !fuse_rest && !sc.fixed() && !sc.is_static() && use_refine_rows()) {
        int tT = 6;
        for (int t = 1; t < 6; t++)
            if (tk.bound[t - 1] >= KTd / 8) {
                tT = t;
                break;
            }
        const int64_t nt = tstart[kTiers] - tstart[tT];
        const double rb = (double)nt * KTd * (wide ? 8.0 : 4.0);
        if (nt > 0 && rb <= kRowsMaxBytes) {
            rt.tfirst = tT;
            rt.nt = (int32_t)nt;
            rt.nsmall = (int32_t)(tstart[6] - tstart[tT]);
            for (int t = tT; t < kTiers; t++) rt.entries += (int64_t)hedge[t];
            GP_TRY(sc.alloc((char **)&rt.rows, (size_t)rb));
            GP_TRY(sc.alloc(&rt.rowidx, n));
            GP_TRY(sc.alloc(&rt.big, (size_t)g.nnz / kRowChunk + (size_t)g.nnz / kRowSplit + 1));
            GP_TRY(sc.alloc(&rt.nbig, 1));
            GP_TRY(sc.alloc(&rt.pushed, 1));
            GP_HIP(hipMemsetAsync(rt.pushed, 0, sizeof(unsigned long long), s));
            GP_HIP(hipMemsetAsync(rt.rows, 0, (size_t)rb, s));
            GP_HIP(hipMemsetAsync(rt.rowidx, 0xFF, sizeof(int32_t) * (size_t)n, s));
            GP_HIP(hipMemsetAsync(rt.nbig, 0, sizeof(int32_t), s));
            hipLaunchKernelGGL(k_rows_index, dim3(grid_for(nt, 256, 8192)), dim3(256), 0, s, verts, tstart[tT], rt.nt,
                               rt.rowidx);
            GP_LAUNCH_CHECK();
            const int32_t *tv = verts + tstart[tT];
            const DenseBig *dbp = nbig > 0 ? &db : nullptr;
            int rc;
            if (wide)
                rc = KTd == 16 ? rows_fill<16, int64_t>(rt, g.xadj, g.adjncy, g.adjwgt, lab8, tv, dbp, dchunks, s)
                   : KTd == 64 ? rows_fill<64, int64_t>(rt, g.xadj, g.adjncy, g.adjwgt, lab8, tv, dbp, dchunks, s)
                               : rows_fill<256, int64_t>(rt, g.xadj, g.adjncy, g.adjwgt, lab8, tv, dbp, dchunks, s);
            else
                rc = KTd == 16 ? rows_fill<16, int32_t>(rt, g.xadj, g.adjncy, g.adjwgt, lab8, tv, dbp, dchunks, s)
                   : KTd == 64 ? rows_fill<64, int32_t>(rt, g.xadj, g.adjncy, g.adjwgt, lab8, tv, dbp, dchunks, s)
                               : rows_fill<256, int32_t>(rt, g.xadj, g.adjncy, g.adjwgt, lab8, tv, dbp, dchunks, s);
            GP_TRY(rc);
            // per table vertex: its row, list entry, label, proposal and weight
            rt.sel_bytes = (double)nt * (KTd * (wide ? 8.0 : 4.0) + 12.0 + (g.vwgt ? 4.0 : 0.0));
        }
    }

    // One round = one fixed launch sequence; the round index and the stop flag
    // live on the device, so the host issues every round without reading
    // anything back. Round 0 also sizes every scratch slot; with
    // GP_ROUND_GRAPHS=1 the sequence is then captured once as a HIP graph and
    // replayed for the later rounds.
    auto emit_round = [&](hipStream_t s) -> int {
#define RT_TRY(expr)             \
    do {                         \
        int _r = (expr);         \
        if (_r < 0) return _r;   \
    } while (0)
        LPArgs a;
        a.xadj = g.xadj;
        a.adjncy = g.adjncy;
        a.adjwgt = g.adjwgt;
        a.vwgt = g.vwgt;
        a.labels = labels;
        a.W = W;
        a.U = U;
        a.dir_alternate = dir_alternate;
        a.prop = prop;
        a.done = &dev->done;
        a.round = &dev->round;
        a.capv = capv;
        a.lab8 = lab8;
        a.act = act;
        a.group = group;
        a.gs = gstate;
        if (act && afirst < n) {
            RT_TRY(compact(ActFlag{verts + afirst, act, &dev->done}, ActEmit{verts, averts, atier, tsh, afirst},
                           n - afirst, nullptr, acount, sc));
            hipLaunchKernelGGL(k_act_bounds, dim3(1), dim3(64), 0, s, atier, acount, ats);
            GP_LAUNCH_CHECK();
        }
        const int tg_end = rt.rows ? rt.tfirst : kTiers;
        const DenseBig *dbr = rt.rows ? nullptr : &db;
        if (dense && wide)
            RT_TRY(launch_dense_any<int64_t>(a, nlabels, tstart, tl, dbr, dchunks, s, tbytes, tg_end));
        else if (dense)
            RT_TRY(launch_dense_any<int32_t>(a, nlabels, tstart, tl, dbr, dchunks, s, tbytes, tg_end));
        else if (wide)
            RT_TRY(launch_proposals<int64_t>(a, verts, tstart, tl, hub_log, hub_off, gkey, (int64_t *)gval, s,
                                             tbytes, false));
        else
            RT_TRY(launch_proposals<int32_t>(a, verts, tstart, tl, hub_log, hub_off, gkey, (int32_t *)gval, s,
                                             tbytes, split_hubs));
        if (rt.rows) {
            const bool av = act != nullptr;
            if (wide)
                RT_TRY((KTd == 16 ? rows_select<16, int64_t>(a, nlabels, tl, rt, kTiers, av, s)
                       : KTd == 64 ? rows_select<64, int64_t>(a, nlabels, tl, rt, kTiers, av, s)
                                   : rows_select<256, int64_t>(a, nlabels, tl, rt, kTiers, av, s)));
            else
                RT_TRY((KTd == 16 ? rows_select<16, int32_t>(a, nlabels, tl, rt, kTiers, av, s)
                       : KTd == 64 ? rows_select<64, int32_t>(a, nlabels, tl, rt, kTiers, av, s)
                                   : rows_select<256, int32_t>(a, nlabels, tl, rt, kTiers, av, s)));
        }
        if (split_hubs) {
            GP_PROF_LAUNCH("k_hub_insert", tbytes[kTiers - 1], s, hipLaunchKernelGGL(k_hub_insert, dim3(nchunks), dim3(kHubBlock), 0, s, a, hp));
            hipLaunchKernelGGL(k_hub_reduce, dim3(nbuckets), dim3(kRedBlock), 0, s, a, hp);
            hipLaunchKernelGGL(k_hub_scan, dim3(grid_for(nslices, 1, 2048)), dim3(256), 0, s, a, hp, nslices);
            hipLaunchKernelGGL(k_hub_decide, dim3(grid_for(nh, 256, 1024)), dim3(256), 0, s, a, hp, nh);
            GP_LAUNCH_CHECK();
        }
        if (act) {
            hipLaunchKernelGGL(k_act_step, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, g.xadj, n, act, prop, dev,
                               nmbig);
            GP_LAUNCH_CHECK();
        }
        if (fuse_rest) {  // small level: the rest of the round in one launch
            hipLaunchKernelGGL(k_round_small, dim3(1), dim3(kFuseBlock), 0, s, prop, (int32_t)n, vbits, key_bits,
                               g.vwgt, W, U, capv, (int32_t)nlabels, labels, lab8, dev);
            GP_LAUNCH_CHECK();
            return GP_OK;
        }
        // compaction of movers (ascending vertex id)
        RT_TRY(compact(MoverFlag{prop, &dev->done}, MoverEmit{prop, mk, mv}, n, nullptr, nmov, sc));
        uint32_t *k1 = mk, *k2 = mk2;
        int32_t *v1 = mv, *v2 = mv2;
        RT_TRY((radix_sort<uint32_t, int32_t>(&k1, &v1, &k2, &v2, n, nmov, key_bits, sc)));
        const unsigned gb = grid_for(n, 256, 8192);
        hipLaunchKernelGGL(k_heads, dim3(gb), dim3(256), 0, s, k1, nmov, headpos);
        GP_LAUNCH_CHECK();
        RT_TRY((scan<int64_t>(MoverWeight{v1, g.vwgt}, StoreIncl{S}, n, nmov, (int64_t *)nullptr, sc)));
        hipLaunchKernelGGL(k_admit, dim3(gb), dim3(256), 0, s, k1, v1, nmov, headpos, S, W, U, capv, labels, lab8, oldlab,
                           dev, group, gstate, act);
        GP_LAUNCH_CHECK();
        if (act) {
            hipLaunchKernelGGL(k_act_mark, dim3(gb), dim3(256), 0, s, v1, oldlab, nmov, g.xadj, g.adjncy, act, renew,
                               mbig, nmbig);
            hipLaunchKernelGGL(k_act_mark_big, dim3(grid_for(g.nnz / kMarkChunk + 1, 1, 4096)), dim3(256), 0, s, mbig,
                               nmbig, g.xadj, g.adjncy, act, renew);
            GP_LAUNCH_CHECK();
        }
        if (nlabels <= kSmallLabels)
            hipLaunchKernelGGL(k_apply_w_small, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, k1, v1, nmov, oldlab,
                               g.vwgt, nlabels, W);
        else
            hipLaunchKernelGGL(k_apply_w, dim3(gb), dim3(256), 0, s, k1, v1, nmov, oldlab, g.vwgt, headpos, S, W);
        GP_LAUNCH_CHECK();
        if (rt.rows) {
            if (wide)
                RT_TRY((KTd == 16 ? rows_update<16, int64_t>(rt, k1, v1, oldlab, nmov, g.xadj, g.adjncy, g.adjwgt, n, g.nnz, s)
                       : KTd == 64 ? rows_update<64, int64_t>(rt, k1, v1, oldlab, nmov, g.xadj, g.adjncy, g.adjwgt, n, g.nnz, s)
                                   : rows_update<256, int64_t>(rt, k1, v1, oldlab, nmov, g.xadj, g.adjncy, g.adjwgt, n, g.nnz, s)));
            else
                RT_TRY((KTd == 16 ? rows_update<16, int32_t>(rt, k1, v1, oldlab, nmov, g.xadj, g.adjncy, g.adjwgt, n, g.nnz, s)
                       : KTd == 64 ? rows_update<64, int32_t>(rt, k1, v1, oldlab, nmov, g.xadj, g.adjncy, g.adjwgt, n, g.nnz, s)
                                   : rows_update<256, int32_t>(rt, k1, v1, oldlab, nmov, g.xadj, g.adjncy, g.adjwgt, n, g.nnz, s)));
        }
        if (group) hipLaunchKernelGGL(k_round_end_groups, dim3(grid_for(ngroups, 256, 1024)), dim3(256), 0, s, gstate, ngroups);
        hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, s, dev);
        GP_LAUNCH_CHECK();
    #undef RT_TRY
        return GP_OK;
    };
    GP_TRY(emit_round(s));
    if (rounds > 1) {
        bool replayed = false;
        if (use_round_graphs() && !prof_blocks_replay() && !sc.is_static()) {
            hipStream_t cs = capture_stream();
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            if (cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                sc.set_stream(cs, true);
                prof_suspend(true);
                const int rc = emit_round(cs);
                prof_suspend(false);
                sc.set_stream(s, false);
                const hipError_t ec = hipStreamEndCapture(cs, &graph);
                if (rc == GP_OK && ec == hipSuccess && graph &&
                    hipGraphInstantiateWithFlags(&exec, graph, 0) == hipSuccess) {
                    for (int32_t r = 1; r < rounds; r++) GP_HIP(hipGraphLaunch(exec, s));
                    replayed = true;
                }
                (void)hipGetLastError();
            }
            if (replayed) GP_HIP(hipStreamSynchronize(s));  // the executable graph is released below
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
        }
        if (!replayed) {
            const ProfSuspend quiet(prof_first_round_only());
            for (int32_t r = 1; r < rounds; r++) GP_TRY(emit_round(s));
        }
    }
    if (out || prof_on()) {
        LPDev h;
        unsigned long long pushed = 0;
        GP_HIP(hipMemcpyAsync(&h, dev, sizeof(LPDev), hipMemcpyDeviceToHost, s));
        if (rt.rows) GP_HIP(hipMemcpyAsync(&pushed, rt.pushed, sizeof(pushed), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        prof_flush();
        if (!out) return GP_OK;
        out->rounds_run = h.rounds_run;
        out->moves = h.total_moves;
        out->visits = act ? h.visits : (int64_t)h.rounds_run * g.nnz;
        out->row_vertices = rt.rows ? rt.nt : 0;
        out->row_entries = rt.rows ? rt.entries : 0;
        out->row_width = rt.rows ? KTd : 0;
        out->row_sum_bytes = rt.rows ? (wide ? 8 : 4) : 0;
        out->row_updates = rt.rows ? (int64_t)pushed : 0;
        out->group_rounds.clear();
        out->group_moves.clear();
        if (group) {
            std::vector<GroupState> hs(ngroups);
            GP_HIP(hipMemcpy(hs.data(), gstate, sizeof(GroupState) * (size_t)ngroups, hipMemcpyDeviceToHost));
            for (const auto &x : hs) {
                out->group_rounds.push_back(x.rounds_run);
                out->group_moves.push_back(x.total);
            }
        }
    }
    return GP_OK;
}

}  // namespace gp
