// batch.hip — many graphs partitioned together, level by level, as one
// disjoint-union graph (a project addition around the multilevel scheme of
// §III; every graph gets exactly the result of its own gp_partition).
//
// Why the union gives the same result per graph: no edge joins two graphs,
// so LP proposals, admissions and contractions never mix graphs; each label
// carries its own graph's capacity; a graph that stopped coarsening is frozen
// (its vertices keep their labels and propose nothing, so contraction copies
// it unchanged to the next level); a graph that went idle for two rounds
// stays idle while others continue, so per-graph round counts are tracked on
// the device. The coarsest level holds every graph's coarsest graph (or an
// identical copy), where one batched initial partition runs; during
// uncoarsening a graph is refined at the top level and at every level below
// its own coarsest level, and only projected through the copies.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <string>

#include "contract.hpp"
#include "initpart.hpp"
#include "prims.hpp"

namespace gp {

namespace {

// Per graph: total vertex weight, largest vertex weight, vertices without
// neighbours. The vertices of one graph are contiguous, so a wave mostly
// lies in one graph and adds its sums with one atomic each.
__global__ void k_graph_sums(const int32_t *xadj, const int32_t *vwgt, const int32_t *gid, int32_t n,
                             unsigned long long *W, unsigned long long *cmax, int32_t *niso) {
    const int lane = lane_id();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v - lane < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = v < n;
        const int32_t q = valid ? gid[v] : 0;
        const unsigned long long c = valid ? (vwgt ? (unsigned long long)vwgt[v] : 1ull) : 0ull;
        wave_add_keyed(W, q, c, valid);
        wave_add_keyed(niso, q, 1, valid && xadj[v + 1] == xadj[v]);
        const uint64_t vm = __ballot(valid);
        const int32_t q0 = __shfl(q, __ffsll((unsigned long long)vm) - 1, kWave);
        if (__ballot(valid && q != q0) == 0) {
            const unsigned long long mx = wave_max(c);
            if (lane == 0) atomicMax(&cmax[q0], mx);
        } else if (valid) {
            atomicMax(&cmax[q], c);
        }
    }
}

// every edge stays inside its graph
__global__ void k_check_cross(const int32_t *rowof, const int32_t *adjncy, const int32_t *gid, int32_t nnz,
                              int32_t *bad) {
    int b = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        b |= gid[rowof[e]] != gid[adjncy[e]];
    if (b) *bad = 1;
}

__global__ void k_batch_labels(const int32_t *xadj, int32_t n, bool skip_isolated, const int32_t *vwgt,
                               const int32_t *gid, const uint8_t *coarsening, const int64_t *ucl, int32_t *labels,
                               int64_t *W, int64_t *capv, uint8_t *frozen) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool off = skip_isolated && xadj[v + 1] == xadj[v];
        const int32_t q = gid[v];
        labels[v] = off ? -1 : (int32_t)v;
        W[v] = off ? 0 : (vwgt ? vwgt[v] : 1);
        capv[v] = ucl[q];
        frozen[v] = coarsening[q] ? 0 : 1;
    }
}

__global__ void k_coarse_gid(const int32_t *f2c, const int32_t *gid, int32_t n, int32_t *gid_c, int32_t *cnt) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = f2c[v];
        if (i < 0) continue;
        gid_c[i] = gid[v];  // all members of a cluster belong to one graph
    }
}

__global__ void k_count_gid(const int32_t *gid, int32_t n, int32_t *cnt) {
    const int lane = lane_id();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v - lane < n; v += (int64_t)gridDim.x * blockDim.x)
        wave_add_keyed(cnt, v < n ? gid[v] : 0, 1, v < n);
}

__global__ void k_frozen_of(const int32_t *gid, int32_t n, const uint8_t *active, uint8_t *frozen) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        frozen[v] = active[gid[v]] ? 0 : 1;
}

__global__ void k_block_caps(const int32_t *kbase, const int64_t *lmax, int32_t G, int64_t *cap) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < G; q += gridDim.x * blockDim.x)
        for (int32_t b = kbase[q]; b < kbase[q + 1]; b++) cap[b] = lmax[q];
}

__global__ void k_row_ends(const int32_t *xadj, const int32_t *voff, int32_t G, int32_t *out) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q <= G; q += gridDim.x * blockDim.x)
        out[q] = xadj[voff[q]];
}

__global__ void k_local_parts(const int32_t *gid, const int32_t *kbase, int32_t n, int32_t *part) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        part[v] -= kbase[gid[v]];
}

// Cut weight per graph. The entries of one graph are contiguous, so a wave
// takes kCutRows x 64 consecutive entries, each lane sums its cut entries of
// one graph at a time, and the wave adds its sum with one atomic when all of
// its lanes ended in the same graph (a few hundred counters would otherwise
// take one atomic per cut entry).
constexpr int kCutRows = 32;
__global__ __launch_bounds__(256) void k_graph_cuts(const int32_t *rowof, const int32_t *adjncy, const int32_t *adjwgt,
                                                    const int32_t *part, const int32_t *gid, int32_t nnz,
                                                    unsigned long long *cut) {
    constexpr int64_t kSpan = (int64_t)kCutRows * kWave;
    const int lane = lane_id();
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t base = wid * kSpan; base < nnz; base += nw * kSpan) {
        int32_t g = -1;
        unsigned long long acc = 0;
        for (int r = 0; r < kCutRows; r++) {
            const int64_t e = base + (int64_t)r * kWave + lane;
            if (e >= nnz) break;
            const int32_t v = rowof[e];
            if (part[v] == part[adjncy[e]]) continue;
            const int32_t gv = gid[v];
            if (gv != g) {
                if (acc) atomicAdd(&cut[g], acc);
                g = gv;
                acc = 0;
            }
            acc += (unsigned long long)(adjwgt ? adjwgt[e] : 1);
        }
        const uint64_t has = __ballot(acc != 0);
        if (!has) continue;
        const int32_t g0 = __shfl(g, __ffsll((unsigned long long)has) - 1, kWave);
        if (__ballot(acc != 0 && g != g0) == 0) {
            const unsigned long long sum = wave_sum(acc);
            if (lane == 0) atomicAdd(&cut[g0], sum);
        } else if (acc) {
            atomicAdd(&cut[g], acc);
        }
    }
}

struct BLevel {
    DevGraph g;
    int32_t *gid = nullptr;   // graph of each vertex
    int32_t *voff = nullptr;  // device [G+1]
    std::vector<int32_t> hvoff;
    int32_t *f2c = nullptr;   // to the next level
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
    }
    float stop() {
        float ms = 0.f;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

int upload_voff(const std::vector<int32_t> &h, int32_t **d, Scratch &sc) {
    GP_TRY(sc.alloc(d, h.size()));
    GP_HIP(hipMemcpyAsync(*d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, sc.stream()));
    return GP_OK;
}

// per-graph directed entry counts of one level
int graph_nnz(const BLevel &L, int32_t G, std::vector<int64_t> &out, Scratch &sc) {
    int32_t *d = nullptr;
    GP_TRY(sc.alloc(&d, (size_t)G + 1));
    hipLaunchKernelGGL(k_row_ends, dim3(grid_for(G + 1, 256, 1024)), dim3(256), 0, sc.stream(), L.g.xadj, L.voff, G,
                       d);
    GP_LAUNCH_CHECK();
    std::vector<int32_t> h(G + 1);
    GP_HIP(hipMemcpyAsync(h.data(), d, sizeof(int32_t) * (G + 1), hipMemcpyDeviceToHost, sc.stream()));
    GP_HIP(hipStreamSynchronize(sc.stream()));
    out.assign(G, 0);
    for (int32_t q = 0; q < G; q++) out[q] = (int64_t)h[q + 1] - h[q];
    return GP_OK;
}

// Level-0 graph without its vertices that have no neighbour, renumbered in
// ascending order (rank[v] = new id); blocks made graph-local.
__global__ void k_compact_graph(int32_t n, const int32_t *xadj, const int32_t *adjncy, const int32_t *adjwgt,
                                const int32_t *vwgt, const int32_t *part, const int32_t *gid, const int32_t *kbase,
                                const int32_t *rank, int32_t nnz, int32_t *xc, int32_t *ac, int32_t *wc, int32_t *vc,
                                int32_t *pc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (xadj[v + 1] == xadj[v]) continue;
        const int32_t r = rank[v];
        xc[r] = xadj[v];
        vc[r] = vwgt ? vwgt[v] : 1;
        pc[r] = part[v] - (gid ? kbase[gid[v]] : 0);
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        ac[e] = rank[adjncy[e]];
        wc[e] = adjwgt ? adjwgt[e] : 1;
    }
}

__global__ void k_local_blocks(int32_t n, const int32_t *part, const int32_t *gid, const int32_t *kbase,
                               int32_t *out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = part[v] - (gid ? kbase[gid[v]] : 0);
}

struct HasNbr {
    const int32_t *xadj;
    __device__ bool operator()(int64_t v) const { return xadj[v + 1] > xadj[v]; }
};
struct RankOf {
    int32_t *rank;
    __device__ void operator()(int64_t v, int32_t pos) const { rank[v] = pos; }
};

}  // namespace

int write_coarsest(const DevGraph &gc, bool level0, const int32_t *P, const int32_t *gid, const int32_t *d_kbase,
                   const std::vector<int32_t> &hvoff, const std::vector<int32_t> &niso, CoarsestOut &co,
                   Scratch &sc) {
    hipStream_t s = sc.stream();
    const int32_t n = gc.n, nnz = gc.nnz, G = (int32_t)hvoff.size() - 1;
    co.nnz = nnz;
    co.voff.assign(G + 1, 0);
    if (!level0) {  // coarse levels carry explicit weights
        GP_HIP(hipMemcpyAsync(co.xadj, gc.xadj, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
        GP_HIP(hipMemcpyAsync(co.adjncy, gc.adjncy, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
        GP_HIP(hipMemcpyAsync(co.adjwgt, gc.adjwgt, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
        GP_HIP(hipMemcpyAsync(co.vwgt, gc.vwgt, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        if (n > 0) {
            hipLaunchKernelGGL(k_local_blocks, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, P, gid, d_kbase,
                               co.part);
            GP_LAUNCH_CHECK();
        }
        co.voff = hvoff;
        return GP_OK;
    }
    int32_t *rank = nullptr, *cnt = nullptr;
    GP_TRY(sc.alloc(&rank, n));
    GP_TRY(sc.alloc(&cnt, 1));
    GP_TRY(compact(HasNbr{gc.xadj}, RankOf{rank}, n, nullptr, cnt, sc));
    if (n > 0) {
        hipLaunchKernelGGL(k_compact_graph, dim3(grid_for(std::max(n, nnz), 256, 65536)), dim3(256), 0, s, n, gc.xadj,
                           gc.adjncy, gc.adjwgt, gc.vwgt, P, gid, d_kbase, rank, nnz, co.xadj, co.adjncy, co.adjwgt,
                           co.vwgt, co.part);
        GP_LAUNCH_CHECK();
    }
    for (int32_t q = 0; q < G; q++) co.voff[q + 1] = co.voff[q] + (hvoff[q + 1] - hvoff[q]) - niso[q];
    const int32_t n0 = co.voff[G];
    GP_HIP(hipMemcpyAsync(co.xadj + n0, &co.nnz, sizeof(int32_t), hipMemcpyHostToDevice, s));
    GP_HIP(hipStreamSynchronize(s));
    return GP_OK;
}

int partition_batch(const DevGraph &g0, int32_t G, const int32_t *voff_host, const int32_t *k_host, double eps,
                    const gp_params *p, int32_t *part_out, gp_result *res, Scratch &sc, CoarsestOut *cout) {
    hipStream_t s = sc.stream();
    Timer t_total(s);
    const int32_t n = g0.n;
    std::vector<int32_t> hk(k_host, k_host + G), hkbase(G + 1, 0);
    for (int32_t q = 0; q < G; q++) hkbase[q + 1] = hkbase[q] + hk[q];
    const int32_t ktot = hkbase[G];

    // ---- level 0: graph ids, per-graph sums, validation
    BLevel L0;
    L0.g = g0;
    L0.hvoff.assign(voff_host, voff_host + G + 1);
    GP_TRY(upload_voff(L0.hvoff, &L0.voff, sc));
    GP_TRY(sc.alloc(&L0.gid, n));
    GP_TRY(graph_ids(G, n, L0.voff, L0.gid, s));
    int32_t *rowof0 = nullptr, *bad = nullptr;
    GP_TRY(sc.alloc(&bad, 1));
    GP_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    if (g0.nnz > 0) {
        GP_TRY(sc.alloc(&rowof0, g0.nnz));
        GP_TRY(build_rowof(g0, rowof0, sc));
        hipLaunchKernelGGL(k_check_cross, dim3(grid_for(g0.nnz, 256, 8192)), dim3(256), 0, s, rowof0, g0.adjncy,
                           L0.gid, g0.nnz, bad);
        GP_LAUNCH_CHECK();
    }
    unsigned long long *dW = nullptr, *dC = nullptr;
    int32_t *dI = nullptr;
    GP_TRY(sc.alloc(&dW, G));
    GP_TRY(sc.alloc(&dC, G));
    GP_TRY(sc.alloc(&dI, G));
    GP_HIP(hipMemsetAsync(dW, 0, sizeof(unsigned long long) * G, s));
    GP_HIP(hipMemsetAsync(dC, 0, sizeof(unsigned long long) * G, s));
    GP_HIP(hipMemsetAsync(dI, 0, sizeof(int32_t) * G, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_graph_sums, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, g0.xadj, g0.vwgt, L0.gid, n,
                           dW, dC, dI);
        GP_LAUNCH_CHECK();
    }
    std::vector<unsigned long long> hW(G), hC(G);
    std::vector<int32_t> hI(G);
    int32_t hbad = 0;
    GP_HIP(hipMemcpyAsync(hW.data(), dW, sizeof(unsigned long long) * G, hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(hC.data(), dC, sizeof(unsigned long long) * G, hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(hI.data(), dI, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    if (hbad) {
        set_error("partition_batch: an edge joins two graphs of the batch");
        return GP_ERR_GRAPH;
    }
    std::vector<int64_t> lmax(G), ucl(G);
    for (int32_t q = 0; q < G; q++) {
        const int64_t W = (int64_t)hW[q], kq = hk[q];
        const int64_t qd = W / kq + (W % kq != 0);
        lmax[q] = (int64_t)std::floor((1.0 + eps) * (double)qd);
        ucl[q] = std::max((int64_t)hC[q], lmax[q] - qd);
    }
    int64_t tw = 0;
    GP_TRY(total_edge_weight(g0, &tw, sc));
    const bool wide = tw >= (int64_t)INT_MAX;
    int64_t *d_ucl = nullptr, *d_lmax = nullptr, *d_bcap = nullptr;
    int32_t *d_kbase = nullptr;
    uint8_t *d_flag = nullptr;
    GP_TRY(sc.alloc(&d_ucl, G));
    GP_TRY(sc.alloc(&d_lmax, G));
    GP_TRY(sc.alloc(&d_bcap, std::max(ktot, 1)));
    GP_TRY(sc.alloc(&d_flag, G));
    GP_TRY(upload_voff(hkbase, &d_kbase, sc));
    GP_HIP(hipMemcpyAsync(d_ucl, ucl.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, s));
    GP_HIP(hipMemcpyAsync(d_lmax, lmax.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_block_caps, dim3(grid_for(G, 256, 1024)), dim3(256), 0, s, d_kbase, d_lmax, G, d_bcap);
    GP_LAUNCH_CHECK();

    // ---- per-graph coarsening state
    std::vector<int64_t> cur(G), ev_c(G, 0), ev_r(G, 0);
    std::vector<int32_t> Lg(G, 0);
    std::vector<uint8_t> coarsening(G);
    for (int32_t q = 0; q < G; q++) {
        cur[q] = (int64_t)(L0.hvoff[q + 1] - L0.hvoff[q]) - hI[q];
        coarsening[q] = cur[q] > (int64_t)p->coarsest_per_k * hk[q];
    }
    std::vector<BLevel> lev;
    lev.push_back(L0);
    Timer t_coarse(s);
    for (;;) {
        bool any = false;
        for (int32_t q = 0; q < G; q++) any |= coarsening[q] != 0;
        if (!any) break;
        const size_t L = lev.size() - 1;
        const BLevel &f = lev[L];
        const bool skip = (L == 0);
        std::vector<int64_t> nnzg;
        GP_TRY(graph_nnz(f, G, nnzg, sc));
        int32_t *labels = nullptr;
        int64_t *W = nullptr, *capv = nullptr;
        uint8_t *frozen = nullptr;
        GP_TRY(sc.alloc(&labels, f.g.n));
        GP_TRY(sc.alloc(&W, f.g.n));
        GP_TRY(sc.alloc(&capv, f.g.n));
        GP_TRY(sc.alloc(&frozen, f.g.n));
        GP_HIP(hipMemcpyAsync(d_flag, coarsening.data(), G, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_batch_labels, dim3(grid_for(f.g.n, 256, 65536)), dim3(256), 0, s, f.g.xadj, f.g.n, skip,
                           f.g.vwgt, f.gid, d_flag, d_ucl, labels, W, capv, frozen);
        GP_LAUNCH_CHECK();
        LPOut st;
        GP_TRY(lp_run(f.g, labels, W, f.g.n, 0, p->rounds_coarsen, p->dir_alternate, wide, &st, sc, capv, frozen,
                      f.gid, G));
        for (int32_t q = 0; q < G; q++)
            if (coarsening[q]) ev_c[q] += (int64_t)st.group_rounds[q] * nnzg[q];
        CoarseOut co;
        GP_TRY(sc.alloc(&co.xadj, (size_t)f.g.n + 1));
        GP_TRY(sc.alloc(&co.adjncy, std::max(f.g.nnz, 1)));
        GP_TRY(sc.alloc(&co.adjwgt, std::max(f.g.nnz, 1)));
        GP_TRY(sc.alloc(&co.vwgt, std::max(f.g.n, 1)));
        GP_TRY(sc.alloc(&co.f2c, std::max(f.g.n, 1)));
        GP_TRY(contract(f.g, labels, skip, co, sc));
        BLevel c;
        c.g.n = co.n;
        c.g.nnz = co.nnz;
        c.g.xadj = co.xadj;
        c.g.adjncy = co.adjncy;
        c.g.adjwgt = co.adjwgt;
        c.g.vwgt = co.vwgt;
        int32_t *cnt = nullptr;
        GP_TRY(sc.alloc(&c.gid, std::max(co.n, 1)));
        GP_TRY(sc.alloc(&cnt, G));
        GP_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * G, s));
        hipLaunchKernelGGL(k_coarse_gid, dim3(grid_for(f.g.n, 256, 65536)), dim3(256), 0, s, co.f2c, f.gid, f.g.n,
                           c.gid, cnt);
        if (co.n > 0)
            hipLaunchKernelGGL(k_count_gid, dim3(grid_for(co.n, 256, 65536)), dim3(256), 0, s, c.gid, co.n, cnt);
        GP_LAUNCH_CHECK();
        std::vector<int32_t> hc(G);
        GP_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        c.hvoff.assign(G + 1, 0);
        for (int32_t q = 0; q < G; q++) c.hvoff[q + 1] = c.hvoff[q] + hc[q];
        GP_TRY(upload_voff(c.hvoff, &c.voff, sc));
        lev[L].f2c = co.f2c;
        lev.push_back(c);
        // per-graph stop rules
        for (int32_t q = 0; q < G; q++) {
            if (!coarsening[q]) continue;
            const int64_t nf = cur[q], nc = hc[q];
            if (nc == nf) {  // did not shrink: the copy at L+1 stands for level L
                Lg[q] = (int32_t)L;
                coarsening[q] = 0;
                continue;
            }
            Lg[q] = (int32_t)L + 1;
            cur[q] = nc;
            if ((int64_t)p->stall_den * nc > (int64_t)p->stall_num * nf) coarsening[q] = 0;
            else if (nc <= (int64_t)p->coarsest_per_k * hk[q]) coarsening[q] = 0;
        }
    }
    const float ms_coarse = t_coarse.stop();

    // ---- batched initial partition on the top level
    Timer t_init(s);
    const size_t T = lev.size() - 1;
    BatchInfo bi;
    bi.G = G;
    bi.voff = lev[T].hvoff;
    bi.k = hk;
    bi.kbase = hkbase;
    bi.lmax = lmax;
    bi.d_voff = lev[T].voff;
    bi.d_kbase = d_kbase;
    bi.d_gid = lev[T].gid;
    bi.d_lmax = d_lmax;
    int32_t *P = nullptr;
    GP_TRY(sc.alloc(&P, std::max(lev[T].g.n, 1)));
    GP_TRY(initial_partition_batch(lev[T].g, T == 0, bi, p->seed, p->attempts, p->rounds_refine, p->dir_alternate,
                                   p->init_fm, wide, P, sc));
    const float ms_init = t_init.stop();
    if (cout) return write_coarsest(lev[T].g, T == 0, P, lev[T].gid, d_kbase, lev[T].hvoff, hI, *cout, sc);

    // ---- uncoarsening: graph q is refined at the top and below its own coarsest level
    Timer t_ref(s);
    int64_t *B = nullptr;
    GP_TRY(sc.alloc(&B, std::max(ktot, 1)));
    uint8_t *frozen = nullptr;
    std::vector<uint8_t> refine(G);
    for (size_t l = T + 1; l-- > 0;) {
        const BLevel &gl = lev[l];
        int32_t *Pl = P;
        if (l < T) {
            if (l == 0) Pl = part_out;
            else GP_TRY(sc.alloc(&Pl, std::max(gl.g.n, 1)));
            GP_TRY(project(gl.g.n, gl.f2c, P, Pl, s));
        } else if (l == 0) {
            GP_HIP(hipMemcpyAsync(part_out, P, sizeof(int32_t) * (size_t)gl.g.n, hipMemcpyDeviceToDevice, s));
            Pl = part_out;
        }
        P = Pl;
        bool any = false;
        for (int32_t q = 0; q < G; q++) {
            refine[q] = (l == T) || ((int32_t)l < Lg[q]);
            any |= refine[q] != 0;
        }
        if (!any || gl.g.n == 0) continue;
        std::vector<int64_t> nnzg;
        GP_TRY(graph_nnz(gl, G, nnzg, sc));
        GP_TRY(sc.alloc(&frozen, gl.g.n));
        GP_HIP(hipMemcpyAsync(d_flag, refine.data(), G, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_frozen_of, dim3(grid_for(gl.g.n, 256, 65536)), dim3(256), 0, s, gl.gid, gl.g.n, d_flag,
                           frozen);
        GP_LAUNCH_CHECK();
        GP_TRY(label_weights(gl.g, Pl, B, ktot, sc));
        LPOut st;
        GP_TRY(lp_run(gl.g, Pl, B, ktot, 0, p->rounds_refine, p->dir_alternate, wide, &st, sc, d_bcap, frozen,
                      gl.gid, G));
        for (int32_t q = 0; q < G; q++)
            if (refine[q]) ev_r[q] += (int64_t)st.group_rounds[q] * nnzg[q];
    }
    const float ms_ref = t_ref.stop();

    // ---- vertices without neighbours, local block ids, per-graph metrics
    std::vector<int32_t> iso_first(G + 1, 0);
    for (int32_t q = 0; q < G; q++) iso_first[q + 1] = iso_first[q] + hI[q];
    int32_t *d_iso_first = nullptr;
    GP_TRY(upload_voff(iso_first, &d_iso_first, sc));
    BatchInfo b0 = bi;
    b0.voff = L0.hvoff;
    b0.d_voff = L0.voff;
    b0.d_gid = L0.gid;
    GP_TRY(label_weights(g0, part_out, B, ktot, sc));
    GP_TRY(fill_isolated_batch(g0, b0, d_iso_first, part_out, B, sc));
    GP_TRY(label_weights(g0, part_out, B, ktot, sc));
    unsigned long long *dcut = nullptr;
    GP_TRY(sc.alloc(&dcut, G));
    GP_HIP(hipMemsetAsync(dcut, 0, sizeof(unsigned long long) * G, s));
    if (g0.nnz > 0) {
        hipLaunchKernelGGL(k_graph_cuts, dim3(grid_for(g0.nnz, 256 * kCutRows, 8192)), dim3(256), 0, s, rowof0, g0.adjncy,
                           g0.adjwgt, part_out, L0.gid, g0.nnz, dcut);
        GP_LAUNCH_CHECK();
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_local_parts, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, L0.gid, d_kbase, n,
                           part_out);
        GP_LAUNCH_CHECK();
    }
    std::vector<int64_t> hB(std::max(ktot, 1));
    std::vector<unsigned long long> hcut(G);
    GP_HIP(hipMemcpyAsync(hB.data(), B, sizeof(int64_t) * ktot, hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(hcut.data(), dcut, sizeof(unsigned long long) * G, hipMemcpyDeviceToHost, s));
    const float ms_total = t_total.stop();
    bool all_bal = true;
    for (int32_t q = 0; q < G; q++) {
        int64_t maxb = 0;
        for (int32_t b = hkbase[q]; b < hkbase[q + 1]; b++) maxb = std::max(maxb, hB[b]);
        all_bal &= maxb <= lmax[q];
        if (!res) continue;
        gp_result &r = res[q];
        r.cut = (int64_t)(hcut[q] / 2);
        r.max_block_w = maxb;
        r.lmax = lmax[q];
        r.ucl = ucl[q];
        r.balanced = maxb <= lmax[q];
        r.levels = Lg[q] + 1;
        r.coarsest_n = (int32_t)cur[q];
        r.n_isolated = hI[q];
        r.edge_visits_cluster = ev_c[q];
        r.edge_visits_refine = ev_r[q];
        r.ms_coarsen = ms_coarse;
        r.ms_init = ms_init;
        r.ms_refine = ms_ref;
        r.ms_total = ms_total;
        r.learned_tried = 0;
        r.learned_kept = 0;
        r.plain_cut_coarsest = -1;
        r.learned_cut_coarsest = -1;
    }
    return all_bal ? GP_OK : GP_WARN_IMBALANCED;
}

}  // namespace gp
