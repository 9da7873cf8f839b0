// contract.hip — contraction (§III-A quotient graph; §IV-A relabelling by a
// prefix sum over used labels), projection (§III-C) and the cut (§II-A).
//
// Contraction is sort based instead of the paper's concurrent hash table:
//   used[L] flags -> exclusive scan -> f2c[v] = id[C[v]], n'
//   c'(i) by integer atomics (exact)
//   every directed fine entry (v,u) with f2c[v] != f2c[u] becomes a 64-bit key
//   (i << bits | j) with its weight; stable LSD radix sort of the keys; equal
//   keys form runs whose weights are summed through an inclusive prefix sum;
//   run heads become the coarse entries (rows and columns ascending), and the
//   row offsets are filled from the run rows.
#include <climits>

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

struct CrossFlag {
    const int32_t *rowof, *adjncy, *f2c;
    __device__ bool operator()(int64_t e) const { return f2c[rowof[e]] != f2c[adjncy[e]]; }
};
struct CrossEmit {
    const int32_t *rowof, *adjncy, *adjwgt, *f2c;
    int bits;
    uint64_t *key;
    int32_t *val;
    __device__ void operator()(int64_t e, int32_t pos) const {
        const uint64_t i = (uint32_t)f2c[rowof[e]], j = (uint32_t)f2c[adjncy[e]];
        key[pos] = (i << bits) | j;
        val[pos] = adjwgt ? adjwgt[e] : 1;
    }
};

struct ValIn {
    const int32_t *w;
    __device__ int64_t operator()(int64_t p) const { return (int64_t)w[p]; }
};
struct InclOut {
    int64_t *S;
    __device__ void operator()(int64_t p, int64_t ex, int64_t v) const { S[p] = ex + v; }
};

struct HeadFlag {
    const uint64_t *key;
    __device__ bool operator()(int64_t p) const { return p == 0 || key[p] != key[p - 1]; }
};
struct HeadEmit {
    int32_t *head;
    __device__ void operator()(int64_t p, int32_t r) const { head[r] = (int32_t)p; }
};

__global__ void k_runs(const uint64_t *key, const int64_t *S, const int32_t *head, const int32_t *nruns,
                       const int32_t *m, int bits, int32_t *adjncy_c, int32_t *adjwgt_c, int32_t *overflow) {
    const int32_t R = *nruns, M = *m;
    const uint64_t jm = (uint64_t(1) << bits) - 1;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p0 = head[r];
        const int32_t p1 = (r + 1 < R) ? head[r + 1] - 1 : M - 1;
        const int64_t sum = S[p1] - (p0 > 0 ? S[p0 - 1] : 0);
        if (sum > INT_MAX) *overflow = 1;
        adjncy_c[r] = (int32_t)(key[p0] & jm);
        adjwgt_c[r] = (int32_t)sum;
    }
}

// xadj_c[i] = first run with row >= i, for i in [0, n']
__global__ void k_row_offsets(const uint64_t *key, const int32_t *head, const int32_t *nruns, const int32_t *nc,
                              int bits, int32_t *xadj_c) {
    const int32_t R = *nruns, N = *nc;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= R;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = (r < R) ? (int64_t)(key[head[r]] >> bits) : (int64_t)N;
        const int64_t prev = (r > 0) ? (int64_t)(key[head[r - 1]] >> bits) : -1;
        for (int64_t i = prev + 1; i <= row; i++) xadj_c[i] = (int32_t)r;
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

int contract(const DevGraph &g, const int32_t *labels, bool skip_isolated, const int32_t *rowof,
             CoarseOut &out, Scratch &sc) {
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
    if (nnz > 0) {
        int32_t *ro = const_cast<int32_t *>(rowof);
        if (!ro) {
            GP_TRY(sc.alloc(&ro, nnz));
            GP_TRY(build_rowof(g, ro, sc));
        }
        const int bits = bits_for(nc > 0 ? nc - 1 : 0) > 0 ? bits_for(nc - 1) : 1;
        uint64_t *k1 = nullptr, *k2 = nullptr;
        int32_t *v1 = nullptr, *v2 = nullptr, *d_m = nullptr, *head = nullptr, *d_runs = nullptr;
        int64_t *S = nullptr;
        GP_TRY(sc.alloc(&k1, nnz));
        GP_TRY(sc.alloc(&k2, nnz));
        GP_TRY(sc.alloc(&v1, nnz));
        GP_TRY(sc.alloc(&v2, nnz));
        GP_TRY(sc.alloc(&d_m, 1));
        GP_TRY(sc.alloc(&d_runs, 1));
        GP_TRY(compact(CrossFlag{ro, g.adjncy, out.f2c}, CrossEmit{ro, g.adjncy, g.adjwgt, out.f2c, bits, k1, v1},
                       nnz, nullptr, d_m, sc));
        int32_t m = 0;
        GP_HIP(hipMemcpyAsync(&m, d_m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        if (m > 0) {
            GP_TRY((radix_sort<uint64_t, int32_t>(&k1, &v1, &k2, &v2, m, nullptr, 2 * bits, sc)));
            GP_TRY(sc.alloc(&S, m));
            GP_TRY(sc.alloc(&head, m));
            GP_TRY((scan<int64_t>(ValIn{v1}, InclOut{S}, m, nullptr, (int64_t *)nullptr, sc)));
            GP_TRY(compact(HeadFlag{k1}, HeadEmit{head}, m, nullptr, d_runs, sc));
            const unsigned gm = grid_for(m, 256, 65536);
            hipLaunchKernelGGL(k_runs, dim3(gm), dim3(256), 0, s, k1, S, head, d_runs, d_m, bits, out.adjncy,
                               out.adjwgt, flags);
            GP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_row_offsets, dim3(gm), dim3(256), 0, s, k1, head, d_runs, d_nc, bits, out.xadj);
            GP_LAUNCH_CHECK();
            GP_HIP(hipMemcpyAsync(&nnz_c, d_runs, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        } else {
            GP_HIP(hipMemsetAsync(out.xadj, 0, sizeof(int32_t) * (size_t)(nc + 1), s));
        }
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
    GP_TRY((scan<int64_t>(CutIn{ro, g.adjncy, g.adjwgt, part}, NoOut{}, g.nnz, nullptr, cut_out, sc)));
    hipLaunchKernelGGL(k_halve, dim3(1), dim3(1), 0, s, cut_out);
    GP_LAUNCH_CHECK();
    return GP_OK;
}

}  // namespace gp
