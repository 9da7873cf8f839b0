// mpnn.hip — the learned initial partition: a three-layer message-passing
// network that proposes the k-way assignment of the coarsest graph (the slot
// of the paper's initial partitioning, §III-B), its training loss and
// hand-written backward pass, and Adam.
//
// Inference is bit-reproducible: weights are used rounded to bfloat16 (nearest,
// ties to even) as binary32 values; every sum is a chain of fused
// multiply-adds in a fixed order (neighbours in CSR order from 0, then inputs
// in index order from the bias, self inputs before aggregated ones); the
// reciprocal of a weighted degree and the two ratio features are formed in
// binary64 and rounded once. Nothing else is fused: contraction is off for
// this file. Training kernels use the same forward; their gradients are
// plain binary32 (atomics in the weight-gradient reductions).
//
// Network (per vertex v):
//   X[v]  = (c(v)/c_max, deg(v)/max_deg, y_8[v][0..15]),
//           y_0 = seeded +-1 probes, y_{t+1}[v] = (y_t[v] + (sum_u w(v,u) y_t[u]) / d(v)) / 2
//   h_l   = ReLU(b_l + Ws_l h_{l-1}[v] + Wn_l m_l[v]),  m_l[v] = (sum_u w(v,u) h_{l-1}[u]) / d(v)
//   z[v]  = bh + Wh h_3[v];  block(v) = argmax z[v] (ties -> lowest)
// d(v) is the weighted degree; a vertex without neighbours keeps y and gets m = 0.
#include <cmath>
#include <utility>

#include "mpnn.hpp"
#include "prims.hpp"

#pragma clang fp contract(off)

namespace gp {

int32_t mpnn_param_count(int32_t k) {
    return (2 * kMpHid * kMpFeat + kMpHid) + 2 * (2 * kMpHid * kMpHid + kMpHid) + kMpHid * k + k;
}

namespace {

constexpr int kMB = 256;  // block size of the network kernels

// splitmix64 (Steele, Lea & Flood 2014): finaliser of x + golden gamma.
__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Round to the nearest bfloat16 (ties to even); NaN stays a quiet NaN.
__global__ void k_bf16(const float *__restrict__ in, float *__restrict__ out, int32_t count) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        uint32_t u = __float_as_uint(in[i]);
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0) u = (u & 0xffff0000u) | 0x00400000u;
        else u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
        out[i] = __uint_as_float(u);
    }
}

// 1/d(v) (binary64 reciprocal rounded once) and the maxima of c and deg.
__global__ void k_vstats(int32_t n, const int32_t *__restrict__ xadj, const int32_t *__restrict__ adjwgt,
                         const int32_t *__restrict__ vwgt, bool active_only, float *__restrict__ rinv,
                         int32_t *__restrict__ mx) {
    int32_t cm = 0, dm = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t b = xadj[v], e = xadj[v + 1];
        int64_t s = e - b;
        if (adjwgt) {
            s = 0;
            for (int32_t i = b; i < e; i++) s += adjwgt[i];
        }
        rinv[v] = s > 0 ? (float)(1.0 / (double)s) : 0.0f;
        if (!active_only || e > b) {
            cm = max(cm, vwgt ? vwgt[v] : 1);
            dm = max(dm, e - b);
        }
    }
    cm = wave_max(cm);
    dm = wave_max(dm);
    if (lane_id() == 0) {
        atomicMax(&mx[0], cm);
        atomicMax(&mx[1], dm);
    }
}

// acc <- fma(w(v,u), X[u][c], acc) over the CSR row [b, e) in order. The
// loads of kUnroll neighbours are issued before their (sequential) FMAs, so a
// high-degree row waits on memory once per group instead of once per edge.
constexpr int kUnroll = 16;
__device__ __forceinline__ float row_fma(int32_t b, int32_t e, const int32_t *__restrict__ adjncy,
                                         const int32_t *__restrict__ adjwgt, const float *__restrict__ X,
                                         int32_t stride, int32_t c, float acc) {
    int32_t q = b;
    for (; q + kUnroll <= e; q += kUnroll) {
        float wv[kUnroll], xv[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            wv[j] = adjwgt ? (float)adjwgt[q + j] : 1.0f;
            xv[j] = X[(int64_t)adjncy[q + j] * stride + c];
        }
#pragma unroll
        for (int j = 0; j < kUnroll; j++) acc = __builtin_fmaf(wv[j], xv[j], acc);
    }
    for (; q < e; q++) acc = __builtin_fmaf(adjwgt ? (float)adjwgt[q] : 1.0f, X[(int64_t)adjncy[q] * stride + c], acc);
    return acc;
}

// Rows above kBigRow entries: one workgroup per row. The workgroup stages a
// chunk of neighbours' values in LDS and the first `cols` threads run the same
// sequential FMA chains as row_fma, fed from LDS, chunk after chunk; a
// lane-per-output thread would otherwise wait on memory for the whole row.
constexpr int kBigRow = 2048;
constexpr int kBigStage = 16384;  // staged floats per chunk (64 KB)

struct BigFlag {
    const int32_t *xadj;
    __device__ bool operator()(int64_t v) const { return xadj[v + 1] - xadj[v] > kBigRow; }
};
struct BigEmit {
    int32_t *big;
    __device__ void operator()(int64_t v, int32_t pos) const { big[pos] = (int32_t)v; }
};

// WALK: out[v][c] = (X[v][c] + acc * rinv[v]) / 2, else out[v][c] = acc * rinv[v]
template <bool WALK>
__global__ __launch_bounds__(256) void k_rows_big(const int32_t *__restrict__ big, const int32_t *__restrict__ nbig,
                                                  int32_t cols, const int32_t *__restrict__ xadj,
                                                  const int32_t *__restrict__ adjncy,
                                                  const int32_t *__restrict__ adjwgt, const float *__restrict__ rinv,
                                                  const float *__restrict__ X, float *__restrict__ out) {
    __shared__ float sx[kBigStage];
    __shared__ float sw[kBigStage / 16];
    __shared__ int32_t su[kBigStage / 16];
    const int32_t chunk = kBigStage / cols;  // cols <= 64: at least 256 neighbours per chunk
    const int32_t nb = *nbig;
    for (int32_t r = blockIdx.x; r < nb; r += gridDim.x) {
        const int32_t v = big[r];
        const int32_t b = xadj[v], e = xadj[v + 1];
        float acc = 0.0f;
        for (int32_t q0 = b; q0 < e; q0 += chunk) {
            const int32_t len = min(chunk, e - q0);
            for (int32_t q = threadIdx.x; q < len; q += 256) {
                su[q] = adjncy[q0 + q];
                sw[q] = adjwgt ? (float)adjwgt[q0 + q] : 1.0f;
            }
            __syncthreads();
            for (int32_t i = threadIdx.x; i < len * cols; i += 256) {
                const int32_t q = i / cols, c = i - q * cols;
                sx[i] = X[(int64_t)su[q] * cols + c];
            }
            __syncthreads();
            if (threadIdx.x < cols)
                for (int32_t q = 0; q < len; q++) acc = __builtin_fmaf(sw[q], sx[q * cols + threadIdx.x], acc);
            __syncthreads();
        }
        if (threadIdx.x < cols) {
            const int64_t i = (int64_t)v * cols + threadIdx.x;
            out[i] = WALK ? (X[i] + acc * rinv[v]) * 0.5f : acc * rinv[v];
        }
    }
}

struct ActiveFlag {
    const int32_t *xadj;
    __device__ bool operator()(int64_t v) const { return xadj[v + 1] > xadj[v]; }
};
struct RankEmit {
    int32_t *rank;
    __device__ void operator()(int64_t v, int32_t pos) const { rank[v] = pos; }
};

// y_0[v][j] = -1 if the top bit of splitmix(splitmix(seed) ^ (16 id + j)) is set, else +1
__global__ void k_probes(int32_t n, uint64_t seed, const int32_t *__restrict__ rank, float *__restrict__ Y) {
    const uint64_t base = splitmix(seed);
    const int64_t N = (int64_t)n * kMpProbe;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i / kMpProbe), j = (int32_t)(i % kMpProbe);
        const uint64_t id = rank ? (uint64_t)rank[v] : (uint64_t)v;
        Y[i] = (splitmix(base ^ (id * kMpProbe + (uint64_t)j)) >> 63) ? -1.0f : 1.0f;
    }
}

// one lazy random-walk step of every probe
__global__ void k_walk(int32_t n, const int32_t *__restrict__ xadj, const int32_t *__restrict__ adjncy,
                       const int32_t *__restrict__ adjwgt, const float *__restrict__ rinv,
                       const float *__restrict__ Yin, float *__restrict__ Yout) {
    const int64_t N = (int64_t)n * kMpProbe;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i / kMpProbe), j = (int32_t)(i % kMpProbe);
        const int32_t b = xadj[v], e = xadj[v + 1];
        if (e - b > kBigRow) continue;  // k_rows_big
        const float acc = row_fma(b, e, adjncy, adjwgt, Yin, kMpProbe, j, 0.0f);
        const float self = Yin[i];
        Yout[i] = e > b ? (self + acc * rinv[v]) * 0.5f : self;
    }
}

__global__ void k_features(int32_t n, const int32_t *__restrict__ xadj, const int32_t *__restrict__ vwgt,
                           const int32_t *__restrict__ mx, const float *__restrict__ Y, float *__restrict__ X) {
    const double cmax = (double)mx[0];
    const int32_t dmax = mx[1];
    const int64_t N = (int64_t)n * kMpFeat;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i / kMpFeat), f = (int32_t)(i % kMpFeat);
        float x;
        if (f == 0) x = (float)((double)(vwgt ? vwgt[v] : 1) / cmax);
        else if (f == 1) x = dmax > 0 ? (float)((double)(xadj[v + 1] - xadj[v]) / (double)dmax) : 0.0f;
        else x = Y[(int64_t)v * kMpProbe + (f - 2)];
        X[i] = x;
    }
}

// M[v][c] = (sum_u w(v,u) H[u][c]) / d(v): threads walk (v, c) pairs, so a
// wavefront reads whole contiguous rows H[u][*] of each neighbour.
__global__ void k_aggregate(int32_t n, int32_t din, const int32_t *__restrict__ xadj,
                            const int32_t *__restrict__ adjncy, const int32_t *__restrict__ adjwgt,
                            const float *__restrict__ rinv, const float *__restrict__ H, float *__restrict__ M) {
    const int64_t N = (int64_t)n * din;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i / din), c = (int32_t)(i % din);
        const int32_t b = xadj[v], e = xadj[v + 1];
        if (e - b > kBigRow) continue;  // k_rows_big
        const float acc = row_fma(b, e, adjncy, adjwgt, H, din, c, 0.0f);
        M[i] = e > b ? acc * rinv[v] : 0.0f;
    }
}

// O[v][o] = act(b[o] + sum_i Ws[o][i] H[v][i] + sum_i Wn[o][i] M[v][i]) with
// the weights staged transposed in LDS (lane o reads consecutive words).
// `dp` lanes (a power of two >= dout) serve one vertex.
template <bool NEIGH, bool RELU>
__global__ __launch_bounds__(kMB) void k_dense(int32_t n, int32_t din, int32_t dout, int32_t dp,
                                               const float *__restrict__ H, const float *__restrict__ M,
                                               const float *__restrict__ Ws, const float *__restrict__ Wn,
                                               const float *__restrict__ bias, float *__restrict__ O) {
    __shared__ float sWs[kMpHid * kMpHid], sWn[NEIGH ? kMpHid * kMpHid : 1], sb[kMpHid];
    for (int32_t t = threadIdx.x; t < din * dout; t += kMB) {
        const int32_t o = t / din, i = t % din;
        sWs[i * dout + o] = Ws[t];
        if (NEIGH) sWn[i * dout + o] = Wn[t];
    }
    for (int32_t t = threadIdx.x; t < dout; t += kMB) sb[t] = bias[t];
    __syncthreads();
    const int32_t o = threadIdx.x % dp, vpb = kMB / dp;
    if (o >= dout) return;
    for (int64_t v = (int64_t)blockIdx.x * vpb + threadIdx.x / dp; v < n; v += (int64_t)gridDim.x * vpb) {
        const float *h = H + v * din;
        float acc = sb[o];
        for (int32_t i = 0; i < din; i++) acc = __builtin_fmaf(sWs[i * dout + o], h[i], acc);
        if (NEIGH) {
            const float *m = M + v * din;
            for (int32_t i = 0; i < din; i++) acc = __builtin_fmaf(sWn[i * dout + o], m[i], acc);
        }
        O[v * dout + o] = RELU ? (acc > 0.0f ? acc : 0.0f) : acc;
    }
}

__global__ void k_argmax(int32_t n, int32_t k, const float *__restrict__ Z, const int32_t *__restrict__ xadj,
                         bool active_only, int32_t *__restrict__ part, int32_t *__restrict__ nonfinite) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float *z = Z + (int64_t)v * k;
        int32_t best = 0;
        bool fin = isfinite(z[0]);
        for (int32_t c = 1; c < k; c++) {
            fin &= isfinite(z[c]);
            if (z[c] > z[best]) best = c;
        }
        if (part) part[v] = best;
        if (nonfinite && !fin && (!active_only || xadj[v + 1] > xadj[v])) atomicOr(nonfinite, 1);
    }
}

// ------------------------------------------------------------------ decoding
// Every vertex ranks the blocks by logit (highest first, ties -> lower block);
// round r offers each unplaced vertex's r-th block, and the offers to block t
// are admitted in ascending vertex id while B[t] + (weight of all offers to t
// up to and including v) <= lmax; leftovers go one by one, ascending, to the
// lightest block.

// pref[v][rank] = block; part[v] = -1 (unplaced) or -2 (takes no part)
__global__ void k_prefs(int32_t n, int32_t k, const float *__restrict__ Z, const int32_t *__restrict__ xadj,
                        bool active_only, uint8_t *__restrict__ pref, int32_t *__restrict__ part) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float *z = Z + (int64_t)v * k;
        for (int32_t c = 0; c < k; c++) {
            const float zc = z[c];
            int32_t rank = 0;
            for (int32_t d = 0; d < k; d++) rank += (z[d] > zc) || (z[d] == zc && d < c);
            pref[(int64_t)v * k + rank] = (uint8_t)c;
        }
        part[v] = (active_only && xadj[v + 1] == xadj[v]) ? -2 : -1;
    }
}

constexpr int kDB = 1024;

// one workgroup per block t: admit round r's offers to t in ascending id
__global__ __launch_bounds__(kDB) void k_decode_round(int32_t n, int32_t k, int32_t r, const uint8_t *__restrict__ pref,
                                                      const int32_t *__restrict__ vwgt, int64_t lmax,
                                                      int64_t *__restrict__ B, int32_t *__restrict__ part) {
    __shared__ int64_t tmp[kDB / kWave + 1];
    const int32_t t = blockIdx.x;
    int64_t run = B[t], admitted = 0;
    for (int32_t base = 0; base < n; base += kDB) {
        const int32_t v = base + threadIdx.x;
        int64_t c = 0;
        // only this workgroup changes part[v] for offers to t in this round
        if (v < n && part[v] == -1 && pref[(int64_t)v * k + r] == t) c = vwgt ? vwgt[v] : 1;
        int64_t total;
        const int64_t excl = block_excl_scan<kDB>(c, tmp, &total);
        const bool ok = c > 0 && run + excl + c <= lmax;
        if (ok) part[v] = t;
        admitted += block_sum<kDB>(ok ? c : (int64_t)0, tmp);
        run += total;
    }
    if (threadIdx.x == 0) B[t] += admitted;
}

// unplaced vertices, ascending, each into the currently lightest block. One
// workgroup reads the assignment in 256-vertex chunks; thread 0 then places
// that chunk's unplaced vertices in order (block weights in LDS).
constexpr int kLeftBlock = 256;
__global__ __launch_bounds__(kLeftBlock) void k_decode_leftover(int32_t n, int32_t k,
                                                                const int32_t *__restrict__ vwgt,
                                                                int64_t *__restrict__ B, int32_t *__restrict__ part) {
    __shared__ int64_t sB[kMpMaxK];
    __shared__ uint8_t sleft[kLeftBlock];
    if (blockIdx.x != 0) return;
    for (int32_t t = threadIdx.x; t < k; t += kLeftBlock) sB[t] = B[t];
    for (int32_t v0 = 0; v0 < n; v0 += kLeftBlock) {
        const int32_t v = v0 + threadIdx.x;
        uint8_t left = 0;
        if (v < n) {
            const int32_t p = part[v];
            if (p == -2) part[v] = 0;  // takes no part: any valid block id
            left = p == -1;
        }
        sleft[threadIdx.x] = left;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int32_t i = 0; i < kLeftBlock; i++) {
                if (!sleft[i]) continue;
                int32_t b = 0;
                for (int32_t t = 1; t < k; t++)
                    if (sB[t] < sB[b]) b = t;
                part[v0 + i] = b;
                sB[b] += vwgt ? vwgt[v0 + i] : 1;
            }
        }
        __syncthreads();
    }
    for (int32_t t = threadIdx.x; t < k; t += kLeftBlock) B[t] = sB[t];
}

// ------------------------------------------------------------------ training

__global__ void k_softmax(int32_t n, int32_t k, const float *__restrict__ Z, float *__restrict__ S) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float *z = Z + (int64_t)v * k;
        float m = z[0];
        for (int32_t c = 1; c < k; c++) m = fmaxf(m, z[c]);
        float s = 0.0f;
        for (int32_t c = 0; c < k; c++) s += __expf(z[c] - m);
        const float inv = 1.0f / s;
        for (int32_t c = 0; c < k; c++) S[(int64_t)v * k + c] = __expf(z[c] - m) * inv;
    }
}

constexpr float kPClip = 1e-6f;

// Edge term of the loss: for every directed edge (v,u), p = <S_v, S_u> and
// BCE against [t_v == t_u], weighted by w(v,u)/Omega. gS[v] collects the
// gradient w.r.t. S_v from both directions of each edge (2 * dl/dp * S_u).
// `kp` lanes (a power of two >= k) serve one vertex.
__global__ __launch_bounds__(kMB) void k_edge_loss(int32_t n, int32_t k, int32_t kp, const int32_t *__restrict__ xadj,
                                                   const int32_t *__restrict__ adjncy,
                                                   const int32_t *__restrict__ adjwgt,
                                                   const int32_t *__restrict__ target, const float *__restrict__ S,
                                                   float inv_omega, float *__restrict__ gS, double *__restrict__ loss) {
    const int32_t c = threadIdx.x % kp, vpb = kMB / kp;
    double lsum = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * vpb + threadIdx.x / kp; v < n; v += (int64_t)gridDim.x * vpb) {
        const float sv = c < k ? S[v * k + c] : 0.0f;
        const int32_t tv = target[v];
        float g = 0.0f, l = 0.0f;
        for (int32_t q = xadj[v]; q < xadj[v + 1]; q++) {
            const int32_t u = adjncy[q];
            const float su = c < k ? S[(int64_t)u * k + c] : 0.0f;
            float p = sv * su;
            for (int32_t d = kp / 2; d > 0; d >>= 1) p += __shfl_xor(p, d, kp);
            const float w = (adjwgt ? (float)adjwgt[q] : 1.0f) * inv_omega;
            const bool y = target[u] == tv;
            const float pc = fminf(fmaxf(p, kPClip), 1.0f - kPClip);
            l += w * -(y ? __logf(pc) : __logf(1.0f - pc));
            const bool inside = p > kPClip && p < 1.0f - kPClip;
            const float dldp = inside ? (y ? -1.0f / pc : 1.0f / (1.0f - pc)) : 0.0f;
            g += 2.0f * w * dldp * su;
        }
        if (c < k) gS[v * k + c] = g;
        if (c == 0) lsum += l;
    }
    lsum = wave_sum(lsum);
    if (lane_id() == 0 && lsum != 0.0) atomicAdd(loss, lsum);
}

// Q[c] = sum_v c(v) S[v][c] (binary64 accumulation)
__global__ __launch_bounds__(kMB) void k_colsum(int32_t n, int32_t k, const float *__restrict__ S,
                                                const int32_t *__restrict__ vwgt, double *__restrict__ Q) {
    __shared__ float part[kMpMaxK];
    for (int32_t t = threadIdx.x; t < k; t += kMB) part[t] = 0.0f;
    __syncthreads();
    const int64_t N = (int64_t)n * k;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(i / k);
        atomicAdd(&part[i % k], S[i] * (vwgt ? (float)vwgt[v] : 1.0f));
    }
    __syncthreads();
    for (int32_t t = threadIdx.x; t < k; t += kMB) atomicAdd(&Q[t], (double)part[t]);
}

// dZ = S * (g - <S, g>) with g = gS + balance term 2 lam k (Q_c/C - 1/k) c(v)/C
__global__ void k_softmax_back(int32_t n, int32_t k, const float *__restrict__ S, const float *__restrict__ gS,
                               const double *__restrict__ Q, double invC, float lam, const int32_t *__restrict__ vwgt,
                               float *__restrict__ dZ) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const float cv = (float)((vwgt ? (double)vwgt[v] : 1.0) * invC);
        float dot = 0.0f;
        for (int32_t c = 0; c < k; c++) {
            const float bal = (float)(2.0 * lam * k * (Q[c] * invC - 1.0 / k));
            const float g = gS[(int64_t)v * k + c] + bal * cv;
            dot += S[(int64_t)v * k + c] * g;
        }
        for (int32_t c = 0; c < k; c++) {
            const float bal = (float)(2.0 * lam * k * (Q[c] * invC - 1.0 / k));
            const float g = gS[(int64_t)v * k + c] + bal * cv;
            dZ[(int64_t)v * k + c] = S[(int64_t)v * k + c] * (g - dot);
        }
    }
}

// dH = dH * [Hout > 0]
__global__ void k_relu_mask(int64_t count, float *__restrict__ dH, const float *__restrict__ Hout) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        if (!(Hout[i] > 0.0f)) dH[i] = 0.0f;
}

constexpr int kWgChunk = 32;
constexpr int kWgMaxE = (kMpHid * (kMpHid + 1) + kMB - 1) / kMB;

// gW[o][i] += sum_v A[v][o] B[v][i]; gb[o] += sum_v A[v][o] (when gb != null).
// A block stages kWgChunk rows of A and B in LDS and keeps its share of the
// dout x (din+1) sums in registers; one atomic per entry per block at the end.
__global__ __launch_bounds__(kMB) void k_wgrad(int32_t n, int32_t dout, int32_t din, const float *__restrict__ A,
                                               const float *__restrict__ B, float *__restrict__ gW,
                                               float *__restrict__ gb) {
    __shared__ float sA[kWgChunk * kMpMaxK], sB[kWgChunk * (kMpHid + 1)];
    const int32_t dc = din + 1, E = dout * dc;
    float acc[kWgMaxE];
#pragma unroll
    for (int r = 0; r < kWgMaxE; r++) acc[r] = 0.0f;
    for (int64_t base = (int64_t)blockIdx.x * kWgChunk; base < n; base += (int64_t)gridDim.x * kWgChunk) {
        const int32_t rows = (int32_t)min<int64_t>(kWgChunk, n - base);
        __syncthreads();
        for (int32_t t = threadIdx.x; t < kWgChunk * dout; t += kMB) {
            const int32_t r = t / dout;
            sA[t] = r < rows ? A[(base + r) * dout + t % dout] : 0.0f;
        }
        for (int32_t t = threadIdx.x; t < kWgChunk * dc; t += kMB) {
            const int32_t r = t / dc, i = t % dc;
            sB[t] = r < rows ? (i < din ? B[(base + r) * din + i] : 1.0f) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kWgMaxE; r++) {
            const int32_t e = threadIdx.x + r * kMB;
            if (e < E) {
                const int32_t o = e / dc, i = e % dc;
                float s = acc[r];
                for (int32_t q = 0; q < kWgChunk; q++) s += sA[q * dout + o] * sB[q * dc + i];
                acc[r] = s;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kWgMaxE; r++) {
        const int32_t e = threadIdx.x + r * kMB;
        if (e < E) {
            const int32_t o = e / dc, i = e % dc;
            if (i < din) atomicAdd(&gW[o * din + i], acc[r]);
            else if (gb) atomicAdd(&gb[o], acc[r]);
        }
    }
}

// out1[v][i] = sum_o W1[o][i] D[v][o]; out2 likewise with W2 (when given).
__global__ __launch_bounds__(kMB) void k_dense_t(int32_t n, int32_t dout, int32_t din, const float *__restrict__ D,
                                                 const float *__restrict__ W1, const float *__restrict__ W2,
                                                 float *__restrict__ out1, float *__restrict__ out2) {
    __shared__ float s1[kMpHid * kMpMaxK], s2[kMpHid * kMpMaxK];
    for (int32_t t = threadIdx.x; t < din * dout; t += kMB) {
        s1[t] = W1[t];
        if (W2) s2[t] = W2[t];
    }
    __syncthreads();
    const int64_t N = (int64_t)n * din;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / din;
        const int32_t i = (int32_t)(t % din);
        const float *d = D + v * dout;
        float a = 0.0f, b = 0.0f;
        for (int32_t o = 0; o < dout; o++) {
            a += s1[o * din + i] * d[o];
            if (W2) b += s2[o * din + i] * d[o];
        }
        out1[t] = a;
        if (W2) out2[t] = b;
    }
}

// out[u][i] += sum_{v in N(u)} w(u,v) dM[v][i] / d(v)   (transpose of the aggregation)
__global__ void k_aggregate_t(int32_t n, int32_t din, const int32_t *__restrict__ xadj,
                              const int32_t *__restrict__ adjncy, const int32_t *__restrict__ adjwgt,
                              const float *__restrict__ rinv, const float *__restrict__ dM, float *__restrict__ out) {
    const int64_t N = (int64_t)n * din;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = (int32_t)(i / din), c = (int32_t)(i % din);
        float acc = 0.0f;
        for (int32_t q = xadj[u]; q < xadj[u + 1]; q++) {
            const int32_t v = adjncy[q];
            acc += (adjwgt ? (float)adjwgt[q] : 1.0f) * rinv[v] * dM[(int64_t)v * din + c];
        }
        out[i] += acc;
    }
}

__global__ void k_adam(int32_t count, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Net {  // offsets of the parameter blocks
    int64_t ws[3], wn[3], b[3], wh, bh;
    explicit Net(int32_t k) {
        int64_t o = 0;
        const int din[3] = {kMpFeat, kMpHid, kMpHid};
        for (int l = 0; l < 3; l++) {
            ws[l] = o;
            o += (int64_t)kMpHid * din[l];
            wn[l] = o;
            o += (int64_t)kMpHid * din[l];
            b[l] = o;
            o += kMpHid;
        }
        wh = o;
        o += (int64_t)kMpHid * k;
        bh = o;
        (void)k;
    }
};

// the rows above kBigRow entries (device list and count)
int big_rows(const DevGraph &g, int32_t **big, int32_t **nbig, Scratch &sc) {
    GP_TRY(sc.alloc(big, g.n));
    GP_TRY(sc.alloc(nbig, 1));
    GP_HIP(hipMemsetAsync(*nbig, 0, sizeof(int32_t), sc.stream()));
    return compact(BigFlag{g.xadj}, BigEmit{*big}, g.n, nullptr, *nbig, sc);
}

struct Acts {  // forward activations kept for the backward pass
    float *X = nullptr, *rinv = nullptr, *H[3] = {}, *M[3] = {}, *Z = nullptr, *Wt = nullptr;
};

int run_forward(const DevGraph &g, int32_t k, const float *params, uint64_t seed, bool active_only, Acts &a,
                Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = g.n, P = mpnn_param_count(k);
    GP_TRY(sc.alloc(&a.X, (size_t)n * kMpFeat));
    GP_TRY(sc.alloc(&a.rinv, n));
    GP_TRY(sc.alloc(&a.Wt, P));
    for (int l = 0; l < 3; l++) {
        GP_TRY(sc.alloc(&a.H[l], (size_t)n * kMpHid));
        GP_TRY(sc.alloc(&a.M[l], (size_t)n * (l == 0 ? kMpFeat : kMpHid)));
    }
    GP_TRY(sc.alloc(&a.Z, (size_t)n * k));
    hipLaunchKernelGGL(k_bf16, dim3(grid_for(P, 256, 256)), dim3(256), 0, s, params, a.Wt, P);
    GP_LAUNCH_CHECK();
    GP_TRY(mpnn_features(g, seed, active_only, a.X, a.rinv, sc));
    const Net net(k);
    const float *in = a.X;
    int32_t *big = nullptr, *nbig = nullptr;
    GP_TRY(big_rows(g, &big, &nbig, sc));
    for (int l = 0; l < 3; l++) {
        const int32_t din = l == 0 ? kMpFeat : kMpHid;
        hipLaunchKernelGGL(k_aggregate, dim3(grid_for((int64_t)n * din, 256, 1 << 16)), dim3(256), 0, s, n, din,
                           g.xadj, g.adjncy, g.adjwgt, a.rinv, in, a.M[l]);
        hipLaunchKernelGGL(k_rows_big<false>, dim3(grid_for(n, 1, 1024)), dim3(256), 0, s, big, nbig, din, g.xadj,
                           g.adjncy, g.adjwgt, a.rinv, in, a.M[l]);
        GP_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_dense<true, true>), dim3(grid_for(n, kMB / kMpHid, 2048)), dim3(kMB), 0, s, n, din,
                           kMpHid, kMpHid, in, a.M[l], a.Wt + net.ws[l], a.Wt + net.wn[l], a.Wt + net.b[l], a.H[l]);
        GP_LAUNCH_CHECK();
        in = a.H[l];
    }
    const int32_t kp = pow2_at_least(k);
    hipLaunchKernelGGL((k_dense<false, false>), dim3(grid_for(n, kMB / kp, 2048)), dim3(kMB), 0, s, n, kMpHid, k, kp,
                       in, nullptr, a.Wt + net.wh, nullptr, a.Wt + net.bh, a.Z);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

}  // namespace

int mpnn_features(const DevGraph &g, uint64_t seed, bool active_only, float *X, float *rinv, Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = g.n;
    if (n == 0) return GP_OK;
    float *r = rinv, *Ya = nullptr, *Yb = nullptr;
    int32_t *mx = nullptr, *rank = nullptr, *cnt = nullptr;
    if (!r) GP_TRY(sc.alloc(&r, n));
    GP_TRY(sc.alloc(&Ya, (size_t)n * kMpProbe));
    GP_TRY(sc.alloc(&Yb, (size_t)n * kMpProbe));
    GP_TRY(sc.alloc(&mx, 2));
    GP_HIP(hipMemsetAsync(mx, 0, sizeof(int32_t) * 2, s));
    hipLaunchKernelGGL(k_vstats, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, n, g.xadj, g.adjwgt, g.vwgt,
                       active_only, r, mx);
    GP_LAUNCH_CHECK();
    if (active_only) {
        GP_TRY(sc.alloc(&rank, n));
        GP_TRY(sc.alloc(&cnt, 1));
        GP_HIP(hipMemsetAsync(rank, 0, sizeof(int32_t) * (size_t)n, s));
        GP_TRY(compact(ActiveFlag{g.xadj}, RankEmit{rank}, n, nullptr, cnt, sc));
    }
    int32_t *big = nullptr, *nbig = nullptr;
    GP_TRY(big_rows(g, &big, &nbig, sc));
    const unsigned gp16 = grid_for((int64_t)n * kMpProbe, 256, 1 << 16);
    hipLaunchKernelGGL(k_probes, dim3(gp16), dim3(256), 0, s, n, seed, rank, Ya);
    GP_LAUNCH_CHECK();
    for (int t = 0; t < kMpWalk; t++) {
        hipLaunchKernelGGL(k_walk, dim3(gp16), dim3(256), 0, s, n, g.xadj, g.adjncy, g.adjwgt, r, Ya, Yb);
        hipLaunchKernelGGL(k_rows_big<true>, dim3(grid_for(n, 1, 1024)), dim3(256), 0, s, big, nbig, kMpProbe,
                           g.xadj, g.adjncy, g.adjwgt, r, Ya, Yb);
        GP_LAUNCH_CHECK();
        std::swap(Ya, Yb);
    }
    hipLaunchKernelGGL(k_features, dim3(grid_for((int64_t)n * kMpFeat, 256, 1 << 16)), dim3(256), 0, s, n, g.xadj,
                       g.vwgt, mx, Ya, X);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

int mpnn_forward(const DevGraph &g, int32_t k, const float *params, uint64_t seed, bool active_only, float *Z,
                 int32_t *part, int32_t *nonfinite_dev, Scratch &sc) {
    if (g.n == 0) return GP_OK;
    Acts a;
    GP_TRY(run_forward(g, k, params, seed, active_only, a, sc));
    hipStream_t s = sc.stream();
    if (Z) GP_HIP(hipMemcpyAsync(Z, a.Z, sizeof(float) * (size_t)g.n * k, hipMemcpyDeviceToDevice, s));
    if (part || nonfinite_dev) {
        hipLaunchKernelGGL(k_argmax, dim3(grid_for(g.n, 256, 4096)), dim3(256), 0, s, g.n, k, a.Z, g.xadj,
                           active_only, part, nonfinite_dev);
        GP_LAUNCH_CHECK();
    }
    return GP_OK;
}

int mpnn_decode(const DevGraph &g, int32_t k, const float *Z, int64_t lmax, bool active_only, int32_t *part,
                Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = g.n;
    if (n == 0) return GP_OK;
    uint8_t *pref = nullptr;
    int64_t *B = nullptr;
    GP_TRY(sc.alloc(&pref, (size_t)n * k));
    GP_TRY(sc.alloc(&B, k));
    GP_HIP(hipMemsetAsync(B, 0, sizeof(int64_t) * (size_t)k, s));
    hipLaunchKernelGGL(k_prefs, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, k, Z, g.xadj, active_only, pref,
                       part);
    GP_LAUNCH_CHECK();
    for (int32_t r = 0; r < k; r++) {
        hipLaunchKernelGGL(k_decode_round, dim3(k), dim3(kDB), 0, s, n, k, r, pref, g.vwgt, lmax, B, part);
        GP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_decode_leftover, dim3(1), dim3(kLeftBlock), 0, s, n, k, g.vwgt, B, part);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

int mpnn_backward(const DevGraph &g, int32_t k, const float *params, uint64_t seed, const int32_t *target,
                  float lam, float *grad, double *loss_host, Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = g.n, P = mpnn_param_count(k);
    GP_HIP(hipMemsetAsync(grad, 0, sizeof(float) * (size_t)P, s));
    if (n == 0) {
        if (loss_host) loss_host[0] = loss_host[1] = 0.0;
        return GP_OK;
    }
    Acts a;
    GP_TRY(run_forward(g, k, params, seed, false, a, sc));
    // Omega (sum of all directed edge weights) and C (total vertex weight)
    int64_t omega = 0;
    GP_TRY(total_edge_weight(g, &omega, sc));
    const int32_t kp = pow2_at_least(k);
    float *S = nullptr, *gS = nullptr, *dZ = nullptr, *dA = nullptr, *dB = nullptr, *dM = nullptr;
    double *acc = nullptr;  // [0] edge loss, [1..k] Q, [k+1] C
    GP_TRY(sc.alloc(&S, (size_t)n * k));
    GP_TRY(sc.alloc(&gS, (size_t)n * k));
    GP_TRY(sc.alloc(&dZ, (size_t)n * k));
    GP_TRY(sc.alloc(&dA, (size_t)n * kMpHid));
    GP_TRY(sc.alloc(&dB, (size_t)n * kMpHid));
    GP_TRY(sc.alloc(&dM, (size_t)n * kMpHid));
    GP_TRY(sc.alloc(&acc, (size_t)k + 2));
    GP_HIP(hipMemsetAsync(acc, 0, sizeof(double) * ((size_t)k + 2), s));
    hipLaunchKernelGGL(k_softmax, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, k, a.Z, S);
    GP_LAUNCH_CHECK();
    const float inv_omega = omega > 0 ? (float)(1.0 / (double)omega) : 0.0f;
    hipLaunchKernelGGL(k_edge_loss, dim3(grid_for(n, kMB / kp, 4096)), dim3(kMB), 0, s, n, k, kp, g.xadj, g.adjncy,
                       g.adjwgt, target, S, inv_omega, gS, acc);
    GP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum, dim3(grid_for((int64_t)n * k, 256, 1024)), dim3(kMB), 0, s, n, k, S, g.vwgt,
                       acc + 1);
    GP_LAUNCH_CHECK();
    // total vertex weight on the host (a single small copy)
    double C = (double)n;
    if (g.vwgt) {
        std::vector<int32_t> hv(n);
        GP_HIP(hipMemcpyAsync(hv.data(), g.vwgt, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        C = 0.0;
        for (int32_t x : hv) C += x;
    }
    hipLaunchKernelGGL(k_softmax_back, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, k, S, gS, acc + 1, 1.0 / C,
                       lam, g.vwgt, dZ);
    GP_LAUNCH_CHECK();
    const Net net(k);
    const unsigned gw = grid_for(n, kWgChunk, 512);
    // head
    hipLaunchKernelGGL(k_wgrad, dim3(gw), dim3(kMB), 0, s, n, k, kMpHid, dZ, a.H[2], grad + net.wh, grad + net.bh);
    GP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_dense_t, dim3(grid_for((int64_t)n * kMpHid, 256, 4096)), dim3(kMB), 0, s, n, k, kMpHid, dZ,
                       a.Wt + net.wh, nullptr, dA, nullptr);
    GP_LAUNCH_CHECK();
    for (int l = 2; l >= 0; l--) {
        const int32_t din = l == 0 ? kMpFeat : kMpHid;
        const float *Hin = l == 0 ? a.X : a.H[l - 1];
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_for((int64_t)n * kMpHid, 256, 8192)), dim3(256), 0, s,
                           (int64_t)n * kMpHid, dA, a.H[l]);
        GP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_wgrad, dim3(gw), dim3(kMB), 0, s, n, kMpHid, din, dA, Hin, grad + net.ws[l],
                           grad + net.b[l]);
        GP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_wgrad, dim3(gw), dim3(kMB), 0, s, n, kMpHid, din, dA, a.M[l], grad + net.wn[l],
                           nullptr);
        GP_LAUNCH_CHECK();
        if (l == 0) break;
        hipLaunchKernelGGL(k_dense_t, dim3(grid_for((int64_t)n * din, 256, 4096)), dim3(kMB), 0, s, n, kMpHid, din,
                           dA, a.Wt + net.ws[l], a.Wt + net.wn[l], dB, dM);
        GP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_aggregate_t, dim3(grid_for((int64_t)n * din, 256, 1 << 16)), dim3(256), 0, s, n, din,
                           g.xadj, g.adjncy, g.adjwgt, a.rinv, dM, dB);
        GP_LAUNCH_CHECK();
        std::swap(dA, dB);
    }
    if (loss_host) {
        std::vector<double> h((size_t)k + 1);
        GP_HIP(hipMemcpyAsync(h.data(), acc, sizeof(double) * ((size_t)k + 1), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        double bal = 0.0;
        for (int32_t c = 0; c < k; c++) {
            const double d = h[1 + c] / C - 1.0 / k;
            bal += d * d;
        }
        loss_host[0] = h[0];
        loss_host[1] = lam * k * bal;
    }
    return GP_OK;
}

int mpnn_adam(float *params, float *m, float *v, const float *grad, int32_t count, int32_t step, float lr, float b1,
              float b2, float eps, hipStream_t s) {
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(count, 256, 1024)), dim3(256), 0, s, count, params, m, v, grad, lr, b1,
                       b2, eps, c1, c2);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

}  // namespace gp
