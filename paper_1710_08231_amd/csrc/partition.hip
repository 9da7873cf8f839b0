// partition.hip — the multilevel driver (§III: coarsen, partition the
// coarsest graph, uncoarsen with refinement) and the C ABI of the library.
//
// Host code only orchestrates: every step of the method runs in the kernels
// of lp.hip, contract.hip and initpart.hip. The host reads back two integers
// per level (coarse n and nnz) and small tier counts; rounds of LP never
// synchronise with the host.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "contract.hpp"
#include "initpart.hpp"
#include "mls.hpp"
#include "mpnn.hpp"
#include "prims.hpp"

namespace gp {

static thread_local std::string g_err;
void set_error(const char *msg) { g_err = msg; }
const char *last_error() { return g_err.c_str(); }
AllocStats &alloc_stats() {
    static AllocStats a;
    return a;
}

namespace {
std::mutex g_arena_mu;
std::map<std::pair<int, hipStream_t>, Arena *> g_arenas;
}  // namespace

Arena *arena_for(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_arena_mu);
    Arena *&a = g_arenas[{dev, s}];
    if (!a) a = new Arena();
    return a;
}

namespace {
struct ProfAcc {
    std::string name;
    int64_t launches = 0;
    double ms = 0, bytes = 0;
};
struct ProfPending {
    std::string name;
    hipEvent_t a, b;
    double bytes;
};
int g_prof = 0;       // GP_PROFILE_* bits
bool g_capturing = false;
std::string g_ctx;   // "cluster L3" etc. (GP_PROFILE_BY_LEVEL)
std::string g_only;  // when non-empty, only launches of this kernel are recorded
std::vector<ProfAcc> g_acc;
std::vector<ProfPending> g_pending;
std::vector<hipEvent_t> g_events;
}  // namespace

bool prof_on() { return g_prof != 0; }
bool prof_wants(const char *name) {
    return (g_prof & (GP_PROFILE_KERNELS | GP_PROFILE_EAGER)) && !g_capturing && (g_only.empty() || g_only == name);
}
bool prof_blocks_replay() { return (g_prof & GP_PROFILE_KERNELS) != 0; }
bool prof_calls() { return (g_prof & GP_PROFILE_CALLS) != 0; }
void prof_suspend(bool on) { g_capturing = on; }
bool prof_first_round_only() { return (g_prof & GP_PROFILE_EAGER) && !(g_prof & GP_PROFILE_KERNELS); }
void prof_context(const char *ctx) { g_ctx = ctx ? ctx : ""; }

hipEvent_t prof_event() {
    if (!g_events.empty()) {
        hipEvent_t e = g_events.back();
        g_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void prof_record(const char *name, hipEvent_t a, hipEvent_t b, double bytes) {
    if ((g_prof & GP_PROFILE_BY_LEVEL) && !g_ctx.empty()) g_pending.push_back({g_ctx + "|" + name, a, b, bytes});
    else g_pending.push_back({name, a, b, bytes});
}

void prof_flush() {
    for (auto &p : g_pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.b);
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        ProfAcc *acc = nullptr;
        for (auto &x : g_acc)
            if (x.name == p.name) acc = &x;
        if (!acc) {
            g_acc.push_back(ProfAcc{p.name});
            acc = &g_acc.back();
        }
        acc->launches++;
        acc->ms += ms;
        acc->bytes += p.bytes;
        g_events.push_back(p.a);
        g_events.push_back(p.b);
    }
    g_pending.clear();
}

namespace {

struct HasEdges {
    const int32_t *xadj;
    __device__ int32_t operator()(int64_t v) const { return xadj[v + 1] > xadj[v] ? 1 : 0; }
};

__global__ void k_identity_labels(const int32_t *xadj, int32_t n, bool skip_isolated, const int32_t *vwgt,
                                  int32_t *labels, int64_t *W) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool off = skip_isolated && xadj[v + 1] == xadj[v];
        labels[v] = off ? -1 : (int32_t)v;
        W[v] = off ? 0 : (vwgt ? vwgt[v] : 1);
    }
}

__global__ void k_graph_stats(const int32_t *xadj, const int32_t *adjncy, const int32_t *vwgt, int32_t n, int32_t nnz,
                              unsigned long long *acc /* [0] sum c, [1] max c, [2] isolated, [3] bad */) {
    unsigned long long s = 0, mx = 0, iso = 0, bad = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = vwgt ? vwgt[v] : 1;
        if (c < 1) bad = 1;
        s += (unsigned long long)(c > 0 ? c : 0);
        mx = (unsigned long long)c > mx ? (unsigned long long)c : mx;
        const int32_t b = xadj[v], e = xadj[v + 1];
        if (e < b || b < 0 || e > nnz) bad = 1;
        iso += (b == e);
    }
    s = wave_sum(s);
    iso = wave_sum(iso);
    mx = wave_max(mx);
    bad = wave_max(bad);
    if (lane_id() == 0) {
        atomicAdd(&acc[0], s);
        atomicMax(&acc[1], mx);
        atomicAdd(&acc[2], iso);
        atomicMax(&acc[3], bad);
    }
}

__global__ void k_check_adj(const int32_t *adjncy, const int32_t *adjwgt, int32_t n, int32_t nnz,
                            unsigned long long *bad) {
    unsigned long long b = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = adjncy[e];
        if (u < 0 || u >= n) b = 1;
        if (adjwgt && adjwgt[e] < 1) b = 1;
    }
    b = wave_max(b);
    if (lane_id() == 0 && b) atomicMax(bad, b);
}

// Full graph validation (GP_VALIDATE=1): a self-loop marks the graph bad, and
// the sums over all entries (v, u, w) of h(v, u, w) and of h(u, v, w) are
// accumulated (mod 2^64, so the order does not matter). A symmetric graph's
// entries are the same multiset read either way, so the sums agree; for an
// asymmetric one they differ unless 64-bit hashes collide. h is the
// splitmix64 finaliser of (v << 32 | u) combined with the weight.
__device__ __forceinline__ unsigned long long sym_hash(uint32_t a, uint32_t b, uint32_t w) {
    unsigned long long z = ((unsigned long long)a << 32 | b) + 0x9E3779B97F4A7C15ull * (1ull + w);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_check_symmetry(const int32_t *xadj, const int32_t *adjncy, const int32_t *adjwgt, int32_t n,
                                 unsigned long long *acc /* [0] sum h(v,u,w), [1] sum h(u,v,w), [2] self-loop */) {
    unsigned long long f = 0, r = 0, loop = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        for (int32_t e = xadj[v]; e < xadj[v + 1]; e++) {
            const uint32_t u = (uint32_t)adjncy[e], w = adjwgt ? (uint32_t)adjwgt[e] : 1u;
            loop |= u == (uint32_t)v;
            f += sym_hash((uint32_t)v, u, w);
            r += sym_hash(u, (uint32_t)v, w);
        }
    }
    f = wave_sum(f);
    r = wave_sum(r);
    loop = wave_max(loop);
    if (lane_id() == 0) {
        atomicAdd(&acc[0], f);
        atomicAdd(&acc[1], r);
        atomicMax(&acc[2], loop);
    }
}

// block ids of the vertices with neighbours must lie in [0, lim); the others may hold -1
__global__ void k_check_blocks(const int32_t *xadj, const int32_t *lab, int32_t n, int32_t lim,
                               unsigned long long *bad) {
    unsigned long long b = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool has = xadj[v + 1] > xadj[v];
        if (lab[v] >= lim || lab[v] < (has ? 0 : -1)) b = 1;
    }
    b = wave_max(b);
    if (lane_id() == 0 && b) atomicMax(bad, b);
}

__global__ void k_check_labels(const int32_t *lab, int32_t n, int32_t lim, unsigned long long *bad) {
    unsigned long long b = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (lab[v] < 0 || lab[v] >= lim) b = 1;
    b = wave_max(b);
    if (lane_id() == 0 && b) atomicMax(bad, b);
}

struct Level {
    DevGraph g;
    int32_t *f2c = nullptr;  // this level -> next level
};


}  // namespace

// Host-side summary of a graph: total vertex weight, max vertex weight,
// isolated count. Also validates offsets, neighbour ids and weights.
struct GraphInfo {
    int64_t W = 0, cmax = 0, niso = 0;
};

int partition_batch(const DevGraph &g0, int32_t G, const int32_t *voff_host, const int32_t *k_host, double eps,
                    const gp_params *p, int32_t *part_out, gp_result *res, Scratch &sc, CoarsestOut *cout);

// GP_VALIDATE=1 in the environment adds the symmetry and self-loop pass.
static bool validating() {
    const char *e = std::getenv("GP_VALIDATE");
    return e && *e && *e != '0';
}

static int graph_info(const DevGraph &g, GraphInfo &gi, Scratch &sc) {
    hipStream_t s = sc.stream();
    unsigned long long *acc = nullptr;
    GP_TRY(sc.alloc(&acc, 5));
    GP_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long) * 5, s));
    if (g.n > 0) {
        hipLaunchKernelGGL(k_graph_stats, dim3(grid_for(g.n, 256, 4096)), dim3(256), 0, s, g.xadj, g.adjncy, g.vwgt,
                           g.n, g.nnz, acc);
        GP_LAUNCH_CHECK();
    }
    if (g.nnz > 0) {
        hipLaunchKernelGGL(k_check_adj, dim3(grid_for(g.nnz, 256, 8192)), dim3(256), 0, s, g.adjncy, g.adjwgt, g.n,
                           g.nnz, acc + 4);
        GP_LAUNCH_CHECK();
    }
    unsigned long long h[5];
    int32_t x0[2] = {0, 0};
    GP_HIP(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(&x0[0], g.xadj, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(&x0[1], g.xadj + g.n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    if (h[3] || h[4] || x0[0] != 0 || x0[1] != g.nnz) {
        set_error("graph: bad offsets, neighbour id out of range, or weight < 1");
        return GP_ERR_GRAPH;
    }
    if (h[0] >= (1ull << 62)) {
        set_error("graph: total vertex weight >= 2^62");
        return GP_ERR_OVERFLOW;
    }
    if (validating() && g.n > 0) {
        unsigned long long *sym = nullptr, hs[3];
        GP_TRY(sc.alloc(&sym, 3));
        GP_HIP(hipMemsetAsync(sym, 0, sizeof(unsigned long long) * 3, s));
        hipLaunchKernelGGL(k_check_symmetry, dim3(grid_for(g.n, 256, 4096)), dim3(256), 0, s, g.xadj, g.adjncy,
                           g.adjwgt, g.n, sym);
        GP_LAUNCH_CHECK();
        GP_HIP(hipMemcpyAsync(hs, sym, sizeof(hs), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        if (hs[2]) {
            set_error("graph: self-loop (GP_VALIDATE)");
            return GP_ERR_GRAPH;
        }
        if (hs[0] != hs[1]) {
            set_error("graph: not symmetric, an entry (v, u, w) has no (u, v, w) (GP_VALIDATE)");
            return GP_ERR_GRAPH;
        }
    }
    gi.W = (int64_t)h[0];
    gi.cmax = (int64_t)h[1];
    gi.niso = (int64_t)h[2];
    return GP_OK;
}

static int check_ws(const void *ws, size_t ws_bytes) {
    if (!ws && ws_bytes) {
        set_error("workspace: ws is NULL but ws_bytes is not 0");
        return GP_ERR_ARG;
    }
    return GP_OK;
}

static int check_graph_args(const gp_graph *g) {
    if (!g) {
        set_error("graph is NULL");
        return GP_ERR_ARG;
    }
    if (g->n < 0 || g->nnz < 0 || !g->xadj || (g->nnz > 0 && !g->adjncy)) {
        set_error("graph: n < 0, nnz < 0 or a required array is NULL");
        return GP_ERR_ARG;
    }
    return GP_OK;
}

static DevGraph dev_graph(const gp_graph *g) {
    DevGraph d;
    d.n = g->n;
    d.nnz = g->nnz;
    d.xadj = g->xadj;
    d.adjncy = g->adjncy;
    d.adjwgt = g->adjwgt;
    d.vwgt = g->vwgt;
    return d;
}

static int check_params(const gp_params *pp, int32_t k, const char *who) {
    if (pp->rounds_coarsen < 0 || pp->rounds_refine < 0 || pp->attempts < 1 || pp->coarsest_per_k < 1 ||
        pp->stall_den < 1 || pp->stall_num < 0 || (pp->init_mode != GP_INIT_PLAIN && pp->init_mode != GP_INIT_LEARNED) ||
        pp->active_set < 0 || pp->active_set > 3 || pp->init_fm < 0) {
        set_error((std::string(who) + ": invalid parameters").c_str());
        return GP_ERR_ARG;
    }
    if (pp->mls < 0 || (pp->mls > 0 && (k > kMlsMaxK || pp->mls_queue < 1 || pp->mls_queue > kMlsMaxQueue ||
                                        pp->mls_batch < 0 || pp->mls_batch > kMlsMaxBatch))) {
        set_error((std::string(who) + ": multi-try local search needs mls >= 0, k <= 256, 1 <= mls_queue <= 64 and "
                                      "0 <= mls_batch <= 65536").c_str());
        return GP_ERR_ARG;
    }
    if (pp->init_mode == GP_INIT_LEARNED && (!pp->mpnn_params || k > kMpMaxK || pp->mpnn_max_n < 0)) {
        set_error((std::string(who) + ": learned initial partition needs mpnn_params, k <= 64 and mpnn_max_n >= 0")
                      .c_str());
        return GP_ERR_ARG;
    }
    return GP_OK;
}

static int check_batch_layout(const gp_graph *g, int32_t G, const int32_t *vtx_off_host, const int32_t *k_host,
                              const char *who) {
    if (vtx_off_host[0] != 0 || vtx_off_host[G] != g->n) {
        set_error((std::string(who) + ": vtx_off must start at 0 and end at n").c_str());
        return GP_ERR_ARG;
    }
    for (int32_t q = 0; q < G; q++)
        if (vtx_off_host[q + 1] < vtx_off_host[q] || k_host[q] < 1) {
            set_error((std::string(who) + ": vtx_off must be non-decreasing and every k >= 1").c_str());
            return GP_ERR_ARG;
        }
    return GP_OK;
}

static int64_t lmax_of(int64_t W, int32_t k, double eps) {
    const int64_t q = W / k + (W % k != 0);
    return (int64_t)std::floor((1.0 + eps) * (double)q);
}

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

// GP_TRACE=1 prints per-level device times to stderr (adds synchronisations).
static bool tracing() {
    static const bool on = [] {
        const char *e = std::getenv("GP_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

// Algorithmic bytes of one LP run (GP_PROFILE_CALLS): per edge visit the
// neighbour id, its weight when present and its label (1 byte in the refining
// runs, which gather a byte copy of the block ids); per vertex and round the
// row offsets, own label and proposal (12 bytes, +4 with vertex weights); per
// admitted move 16 bytes (mover record, label write, two weight updates).
// With connection rows (refinement) a table vertex's edges are gathered once,
// to fill its row; every round then reads its row (row_width sums), and each
// admitted mover's edge is pushed into the rows: neighbour id, weight, the
// neighbour's row index, and the two sums it changes.
static double lp_run_bytes(const DevGraph &g, const LPOut &st, bool refine) {
    const double per_edge = 4.0 + (g.adjwgt ? 4.0 : 0.0) + (refine ? 1.0 : 4.0);
    const double per_vertex = 12.0 + (g.vwgt ? 4.0 : 0.0);
    double b = (double)st.rounds_run * g.n * per_vertex + (double)st.moves * 16.0;
    if (st.row_vertices == 0) return b + (double)st.visits * per_edge;
    // (active-set rounds count only the evaluated vertices' edges: then a bound)
    const double gathered = std::max(0.0, (double)st.visits - (double)st.rounds_run * (double)st.row_entries);
    b += (gathered + (double)st.row_entries) * per_edge;
    b += (double)st.rounds_run * (double)st.row_vertices * st.row_width * st.row_sum_bytes;
    b += (double)st.row_updates * (4.0 + (g.adjwgt ? 4.0 : 0.0) + 4.0 + 2.0 * st.row_sum_bytes);
    return b;
}

// Algorithmic bytes of one contraction: the fine graph read once (row
// offsets, labels, neighbour ids, edge and vertex weights when present), the
// coarse id of every entry's neighbour gathered, f2c written, and the coarse
// graph written (row offsets, vertex weights, columns and weights).
static double contract_bytes(const DevGraph &g, const CoarseOut &co) {
    const double fine = 4.0 * (double)g.n * (3.0 + (g.vwgt ? 1.0 : 0.0)) +
                        (double)g.nnz * (8.0 + (g.adjwgt ? 4.0 : 0.0));
    const double coarse = 8.0 * (double)co.n + 8.0 * (double)co.nnz;
    return fine + coarse;
}

// Brackets one LP run (or contraction) of the driver with events when GP_PROFILE_CALLS is on.
struct CallProf {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    CallProf(hipStream_t st, const char *phase, size_t level) : s(st) {
        char ctx[48];
        std::snprintf(ctx, sizeof ctx, "%s L%zu", phase, level);
        prof_context(ctx);
        if (prof_calls()) {
            a = prof_event();
            b = prof_event();
            (void)hipEventRecord(a, s);
        }
    }
    void done(const char *name, double bytes) {
        if (a) {
            (void)hipEventRecord(b, s);
            prof_record(name, a, b, bytes);
            a = nullptr;
        }
        prof_context(nullptr);
    }
};

static int do_partition(const gp_graph *gin, int32_t k, double eps, const gp_params *p, int32_t *part_out,
                        gp_result *res, void *ws, size_t ws_bytes, hipStream_t s, CoarsestOut *cout = nullptr) {
    Scratch sc(s, ws, ws_bytes);
    Timer t_total(s);
    const auto host_t0 = std::chrono::steady_clock::now();
    const AllocStats alloc0 = alloc_stats();
    const DevGraph g0 = dev_graph(gin);
    GraphInfo gi;
    GP_TRY(graph_info(g0, gi, sc));
    const int64_t lmax = lmax_of(gi.W, k, eps);
    const int64_t ceil_wk = gi.W / k + (gi.W % k != 0);
    const int64_t ucl = std::max(gi.cmax, lmax - ceil_wk);
    int64_t tw = 0;
    GP_TRY(total_edge_weight(g0, &tw, sc));
    const bool wide = tw >= (int64_t)INT_MAX;

    std::vector<Level> lev;
    lev.push_back(Level{g0, nullptr});
    int32_t *rowof0 = nullptr;
    if (g0.nnz > 0) {
        GP_TRY(sc.alloc(&rowof0, g0.nnz));
        GP_TRY(build_rowof(g0, rowof0, sc));
    }
    int64_t ev_c = 0, ev_r = 0;
    int64_t cur_n = g0.n - gi.niso;

    // ---- coarsening
    Timer t_coarse(s);
    while (cur_n > (int64_t)p->coarsest_per_k * k) {
        const size_t L = lev.size() - 1;
        const DevGraph &f = lev[L].g;
        const bool skip = (L == 0);
        int32_t *labels = nullptr;
        int64_t *W = nullptr;
        GP_TRY(sc.alloc(&labels, f.n));
        GP_TRY(sc.alloc(&W, f.n));
        hipLaunchKernelGGL(k_identity_labels, dim3(grid_for(f.n, 256, 65536)), dim3(256), 0, s, f.xadj, f.n, skip,
                           f.vwgt, labels, W);
        GP_LAUNCH_CHECK();
        LPOut st;
        Timer t_lp(s);
        CallProf cp(s, "cluster", L);
        GP_TRY(lp_run(f, labels, W, f.n, ucl, p->rounds_coarsen, p->dir_alternate, wide, &st, sc, nullptr, nullptr,
                      nullptr, 0, (p->active_set & 1) != 0));
        cp.done("lp_cluster", lp_run_bytes(f, st, false));
        const float ms_lp = t_lp.stop();
        ev_c += st.visits;
        CoarseOut co;
        GP_TRY(sc.alloc(&co.xadj, (size_t)f.n + 1));
        GP_TRY(sc.alloc(&co.adjncy, f.nnz));
        GP_TRY(sc.alloc(&co.adjwgt, f.nnz));
        GP_TRY(sc.alloc(&co.vwgt, f.n));
        GP_TRY(sc.alloc(&co.f2c, f.n));
        Timer t_ct(s);
        CallProf cpc(s, "contract", L);
        GP_TRY(contract(f, labels, skip, co, sc));
        cpc.done("contract", contract_bytes(f, co));
        if (tracing())
            std::fprintf(stderr, "[gp] level %zu n=%d nnz=%d cluster %.3f ms (%d rounds, %.1f Gvisits/s) "
                                 "contract %.3f ms -> n=%d nnz=%d\n",
                         L, f.n, f.nnz, ms_lp, st.rounds_run,
                         (double)st.rounds_run * f.nnz / (ms_lp * 1e6), t_ct.stop(), co.n, co.nnz);
        if (co.n == cur_n) break;  // no shrink: drop the level
        lev[L].f2c = co.f2c;
        DevGraph c;
        c.n = co.n;
        c.nnz = co.nnz;
        c.xadj = co.xadj;
        c.adjncy = co.adjncy;
        c.adjwgt = co.adjwgt;
        c.vwgt = co.vwgt;
        lev.push_back(Level{c, nullptr});
        const int64_t prev = cur_n;
        cur_n = co.n;
        if ((int64_t)p->stall_den * cur_n > (int64_t)p->stall_num * prev) break;
    }
    const float ms_coarse = t_coarse.stop();

    // ---- initial partition of the coarsest graph, with the learned proposal
    // (the network's argmax) judged against the plain tries when asked for
    Timer t_init(s);
    const size_t Lc = lev.size() - 1;
    const DevGraph &gc = lev[Lc].g;
    const int32_t nc_active = Lc == 0 ? (int32_t)(g0.n - gi.niso) : gc.n;
    int32_t *P = nullptr, *prop = nullptr;
    GP_TRY(sc.alloc(&P, gc.n));
    const bool tried = p->init_mode == GP_INIT_LEARNED && nc_active > 0 && nc_active <= p->mpnn_max_n;
    if (tried) {
        int32_t *nf = nullptr, hnf = 0;
        float *Z = nullptr;
        GP_TRY(sc.alloc(&prop, gc.n));
        GP_TRY(sc.alloc(&Z, (size_t)gc.n * k));
        GP_TRY(sc.alloc(&nf, 1));
        GP_HIP(hipMemsetAsync(nf, 0, sizeof(int32_t), s));
        GP_TRY(mpnn_forward(gc, k, p->mpnn_params, p->mpnn_seed, Lc == 0, Z, nullptr, nf, sc));
        GP_HIP(hipMemcpyAsync(&hnf, nf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
        if (hnf) prop = nullptr;  // a non-finite logit discards the proposal
        else GP_TRY(mpnn_decode(gc, k, Z, lmax, Lc == 0, prop, sc));
    }
    ProposalOut po;
    prof_context("init");
    GP_TRY(initial_partition(gc, Lc == 0, k, lmax, p->seed, p->attempts, p->rounds_refine, p->dir_alternate,
                             p->init_fm, wide, P, sc, prop, prop ? &po : nullptr));
    prof_context(nullptr);
    int64_t plain_cut_c = -1, prop_cut_c = -1;
    int32_t kept = 0;
    if (prop) {
        plain_cut_c = po.plain_cut[0];
        prop_cut_c = po.prop_cut[0];
        kept = po.kept[0];
    } else if (tried) {
        int32_t *rowc = nullptr;
        int64_t *dcut = nullptr;
        GP_TRY(sc.alloc(&rowc, gc.nnz));
        GP_TRY(sc.alloc(&dcut, 1));
        if (gc.nnz > 0) GP_TRY(build_rowof(gc, rowc, sc));
        GP_TRY(cut_dev(gc, P, rowc, dcut, sc));
        GP_HIP(hipMemcpyAsync(&plain_cut_c, dcut, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GP_HIP(hipStreamSynchronize(s));
    }
    const float ms_init = t_init.stop();
    if (tracing()) std::fprintf(stderr, "[gp] initial partition n=%d nnz=%d %.3f ms\n", gc.n, gc.nnz, ms_init);
    if (cout) {
        GP_TRY(write_coarsest(gc, Lc == 0, P, nullptr, nullptr, {0, gc.n}, {(int32_t)gi.niso}, *cout, sc));
        sc.release();
        GP_HIP(hipStreamSynchronize(s));
        return GP_OK;
    }

    // ---- uncoarsening
    Timer t_ref(s);
    int64_t *B = nullptr;
    GP_TRY(sc.alloc(&B, k));
    // level 0 keeps the vertices without neighbours: the search's hash order
    // takes each vertex's rank among the others (its id on the graph without them)
    int32_t *rank0 = nullptr;
    int64_t mls_gain = 0;
    if (p->mls > 0 && gi.niso > 0) {
        GP_TRY(sc.alloc(&rank0, g0.n));
        GP_TRY((scan<int32_t>(HasEdges{g0.xadj}, StoreExcl<int32_t>{rank0}, g0.n, nullptr, (int32_t *)nullptr, sc)));
    }
    for (size_t l = Lc + 1; l-- > 0;) {
        const DevGraph &gl = lev[l].g;
        int32_t *Pl = P;
        if (l < Lc) {
            if (l == 0) Pl = part_out;
            else GP_TRY(sc.alloc(&Pl, gl.n));
            GP_TRY(project(gl.n, lev[l].f2c, P, Pl, s));
        } else if (l == 0) {
            GP_HIP(hipMemcpyAsync(part_out, P, sizeof(int32_t) * (size_t)gl.n, hipMemcpyDeviceToDevice, s));
            Pl = part_out;
        }
        GP_TRY(label_weights(gl, Pl, B, k, sc));
        LPOut st;
        Timer t_lp(s);
        CallProf cp(s, "refine", l);
        GP_TRY(lp_run(gl, Pl, B, k, lmax, p->rounds_refine, p->dir_alternate, wide, &st, sc, nullptr, nullptr, nullptr,
                      0, (p->active_set & 2) != 0));
        cp.done("lp_refine", lp_run_bytes(gl, st, k <= 256));
        if (p->mls > 0) {
            MlsOut mo;
            GP_TRY(mls_refine(gl, k, lmax, Pl, B, l == 0 ? rank0 : nullptr, p->seed, p->mls,
                              p->mls_batch > 0 ? p->mls_batch : 1, p->mls_queue, 50, 0.1, &mo, sc));
            mls_gain += mo.gain;
        }
        if (tracing()) {
            const float ms = t_lp.stop();
            std::fprintf(stderr, "[gp] refine level %zu n=%d nnz=%d %.3f ms (%d rounds, %lld moves, %.1f Gvisits/s)\n",
                         l, gl.n, gl.nnz, ms, st.rounds_run, (long long)st.moves, (double)st.visits / (ms * 1e6));
        }
        ev_r += st.visits;
        P = Pl;
    }
    const float ms_ref = t_ref.stop();

    // ---- vertices without neighbours, final metrics
    GP_TRY(label_weights(g0, part_out, B, k, sc));
    int32_t niso = 0;
    GP_TRY(fill_isolated(g0, k, part_out, B, &niso, sc));
    GP_TRY(label_weights(g0, part_out, B, k, sc));
    int64_t *dcut = nullptr;
    GP_TRY(sc.alloc(&dcut, 1));
    GP_TRY(cut_dev(g0, part_out, rowof0, dcut, sc));
    std::vector<int64_t> hB(k);
    int64_t cut = 0;
    GP_HIP(hipMemcpyAsync(hB.data(), B, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    GP_HIP(hipMemcpyAsync(&cut, dcut, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    const float ms_total = t_total.stop();
    if (tracing()) {
        const AllocStats &a = alloc_stats();
        std::fprintf(stderr, "[gp] partition device %.3f ms, host %.3f ms; %lld allocations (%.1f MB) took %.3f ms of host time; scratch high-water %.1f MB\n",
                     ms_total,
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host_t0).count(),
                     (long long)(a.calls - alloc0.calls), (a.bytes - alloc0.bytes) / 1e6, a.host_ms - alloc0.host_ms,
                     sc.high_water() / 1e6);
    }
    int64_t maxb = 0;
    for (int b = 0; b < k; b++) maxb = std::max(maxb, hB[b]);
    if (res) {
        res->cut = cut;
        res->max_block_w = maxb;
        res->lmax = lmax;
        res->ucl = ucl;
        res->balanced = maxb <= lmax;
        res->levels = (int32_t)lev.size();
        res->coarsest_n = Lc == 0 ? (int32_t)(g0.n - gi.niso) : lev[Lc].g.n;
        res->n_isolated = niso;
        res->edge_visits_cluster = ev_c;
        res->edge_visits_refine = ev_r;
        res->ms_coarsen = ms_coarse;
        res->ms_init = ms_init;
        res->ms_refine = ms_ref;
        res->ms_total = ms_total;
        res->learned_tried = tried;
        res->learned_kept = kept;
        res->plain_cut_coarsest = plain_cut_c;
        res->learned_cut_coarsest = prop_cut_c;
        res->mls_gain = mls_gain;
        res->workspace_bytes = (int64_t)sc.high_water();
    }
    sc.release();
    GP_HIP(hipStreamSynchronize(s));
    return maxb <= lmax ? GP_OK : GP_WARN_IMBALANCED;
}

}  // namespace gp

using namespace gp;

// ---------------------------------------------------------------- static scratch
// The scratch of gp_lp_refine_static: one array per GPU the library runs on
// (the code object's copy on that device), held until the process ends. Host
// code never uses the array's name as an address: its device address is taken
// once per device with hipGetSymbolAddress and kept in g_static_ptr.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::mutex g_static_mu;
static void *g_static_ptr[256];

static int static_scratch(void **out) {
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) {
        set_error("static scratch: device index out of range");
        return GP_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        GP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("static scratch: hipGetSymbolAddress returned NULL");
            return GP_ERR_HIP;
        }
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return GP_OK;
}

// gp_lp_refine's body on a given scratch. A static scratch (sc.is_static())
// also means no HIP events: ms is then the host time of the call.
static int lp_refine_call(const gp_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t flags,
                          int32_t *part_inout, gp_lp_stats *st_host, Scratch &sc, hipStream_t stream) {
    if (k < 1 || lmax < 1 || rounds < 0 || !part_inout || (flags & ~(GP_LP_DIR_ALTERNATE | GP_LP_ACTIVE_SET))) {
        set_error("lp_refine: k < 1, lmax < 1, rounds < 0, part is NULL or unknown flags");
        return GP_ERR_ARG;
    }
    const auto host_t0 = std::chrono::steady_clock::now();
    std::unique_ptr<Timer> t;
    if (!sc.is_static()) t.reset(new Timer(stream));
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    unsigned long long *bad = nullptr;
    GP_TRY(sc.alloc(&bad, 1));
    GP_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), stream));
    if (d.n > 0) {
        hipLaunchKernelGGL(k_check_labels, dim3(grid_for(d.n, 256, 4096)), dim3(256), 0, stream, part_inout, d.n, k,
                           bad);
        GP_LAUNCH_CHECK();
    }
    unsigned long long hb = 0;
    GP_HIP(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, stream));
    GP_HIP(hipStreamSynchronize(stream));
    if (hb) {
        set_error("lp_refine: a block id is outside [0, k)");
        return GP_ERR_GRAPH;
    }
    int64_t tw = 0;
    GP_TRY(total_edge_weight(d, &tw, sc));
    int64_t *W = nullptr;
    GP_TRY(sc.alloc(&W, k));
    GP_TRY(label_weights(d, part_inout, W, k, sc));
    LPOut o;
    GP_TRY(lp_run(d, part_inout, W, k, lmax, rounds, (flags & GP_LP_DIR_ALTERNATE) ? 1 : 0, tw >= (int64_t)INT_MAX, &o,
                  sc, nullptr, nullptr, nullptr, 0, (flags & GP_LP_ACTIVE_SET) != 0));
    const float ms = t ? t->stop()
                       : (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host_t0)
                             .count();
    if (st_host) {
        st_host->rounds_run = o.rounds_run;
        st_host->moves = o.moves;
        st_host->edge_visits = o.visits;
        st_host->ms = ms;
        st_host->workspace_bytes = (int64_t)sc.high_water();
    }
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

extern "C" {

size_t gp_workspace_bytes(int32_t op, int32_t n, int32_t nnz, int32_t k, int32_t flags) {
    if (n < 0 || nnz < 0 || (op == GP_OP_LP_REFINE && k < 1) ||
        (flags & ~(GP_LP_DIR_ALTERNATE | GP_LP_ACTIVE_SET))) {
        set_error("workspace_bytes: n < 0, nnz < 0, k < 1 or unknown flags");
        return 0;
    }
    auto R = [](double x) { return (size_t)((((size_t)(x > 1 ? x : 1)) + 255) & ~(size_t)255); };
    const int64_t m = std::max<int64_t>(std::max<int64_t>(n, nnz), 1);
    // validation counters, the label check, the edge-weight total and its scan temporaries
    const size_t entry = 4 * R(40) + R(8) + (size_t)(6.25 * 2 * 8 * 4 * std::ceil((double)m / kScanTile)) + 65536;
    const bool active = (flags & GP_LP_ACTIVE_SET) != 0;
    switch (op) {
        case GP_OP_LP_CLUSTER: return entry + R(8.0 * n) + lp_scratch_bound(n, nnz, n, active);
        case GP_OP_LP_REFINE: return entry + R(8.0 * k) + lp_scratch_bound(n, nnz, k, active);
        case GP_OP_CONTRACT: return entry + contract_scratch_bound(n, nnz);
        case GP_OP_CUT:
            return entry + R(8) + R(4.0 * nnz) + (size_t)(6.25 * 2 * 4 * 2 * std::ceil((double)m / 256)) + 65536;
        default:
            set_error("workspace_bytes: unknown op (the multilevel calls report theirs in gp_result.workspace_bytes)");
            return 0;
    }
}

void gp_default_params(gp_params *p) {
    if (!p) return;
    p->rounds_coarsen = 10;
    p->rounds_refine = 25;
    p->coarsest_per_k = 60;
    p->attempts = 4;
    p->stall_num = 19;
    p->stall_den = 20;
    p->dir_alternate = 1;
    p->seed = 0;
    p->init_mode = GP_INIT_PLAIN;
    p->mpnn_max_n = 131072;
    p->mpnn_seed = 0;
    p->mpnn_params = nullptr;
    p->active_set = 0;
    p->init_fm = 0;
    p->mls = 0;
    p->mls_batch = 0;
    p->mls_queue = kMlsMaxQueue;
}

int64_t gp_lmax(int64_t total_vwgt, int32_t k, double eps) {
    if (k < 1 || total_vwgt < 0 || !(eps >= 0.0)) return -1;
    return lmax_of(total_vwgt, k, eps);
}

int gp_lp_cluster(const gp_graph *g, int64_t U, int32_t rounds, int32_t flags, int32_t *labels_out,
                  gp_lp_stats *st_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (U < 1 || rounds < 0 || !labels_out || (flags & ~(GP_LP_DIR_ALTERNATE | GP_LP_ACTIVE_SET))) {
        set_error("lp_cluster: U < 1, rounds < 0, labels_out is NULL or unknown flags");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    Timer t(stream);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    int64_t tw = 0;
    GP_TRY(total_edge_weight(d, &tw, sc));
    int64_t *W = nullptr;
    GP_TRY(sc.alloc(&W, d.n));
    if (d.n > 0) {
        hipLaunchKernelGGL(k_identity_labels, dim3(grid_for(d.n, 256, 65536)), dim3(256), 0, stream, d.xadj, d.n,
                           false, d.vwgt, labels_out, W);
        GP_LAUNCH_CHECK();
    }
    LPOut o;
    GP_TRY(lp_run(d, labels_out, W, d.n, U, rounds, (flags & GP_LP_DIR_ALTERNATE) ? 1 : 0, tw >= (int64_t)INT_MAX, &o,
                  sc, nullptr, nullptr, nullptr, 0, (flags & GP_LP_ACTIVE_SET) != 0));
    const float ms = t.stop();
    if (st_host) {
        st_host->rounds_run = o.rounds_run;
        st_host->moves = o.moves;
        st_host->edge_visits = o.visits;
        st_host->ms = ms;
        st_host->workspace_bytes = (int64_t)sc.high_water();
    }
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_lp_refine(const gp_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t flags,
                 int32_t *part_inout, gp_lp_stats *st_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    Scratch sc(stream, ws, ws_bytes);
    return lp_refine_call(g, k, lmax, rounds, flags, part_inout, st_host, sc, stream);
}

int gp_lp_refine_static(const gp_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t flags,
                        int32_t *part_inout, gp_lp_stats *st_host, hipStream_t stream) {
    GP_TRY(check_graph_args(g));
    if (k < 1 || (flags & ~(GP_LP_DIR_ALTERNATE | GP_LP_ACTIVE_SET))) {
        set_error("lp_refine_static: k < 1 or unknown flags");
        return GP_ERR_ARG;
    }
    const size_t need = gp_workspace_bytes(GP_OP_LP_REFINE, g->n, g->nnz, k, flags);
    if (need == 0 || need > kStaticScratchBytes) {
        set_error((std::string("lp_refine_static: a graph of ") + std::to_string(g->n) + " vertices and " +
                   std::to_string(g->nnz) + " entries with k = " + std::to_string(k) + " may need " +
                   std::to_string(need) + " bytes of scratch; the static scratch holds " +
                   std::to_string(kStaticScratchBytes) + " (use gp_lp_refine with a workspace)").c_str());
        return GP_ERR_WORKSPACE;
    }
    void *ptr = nullptr;
    GP_TRY(static_scratch(&ptr));
    Scratch sc(stream, ptr, kStaticScratchBytes);
    sc.set_static();
    return lp_refine_call(g, k, lmax, rounds, flags, part_inout, st_host, sc, stream);
}

int gp_mls_refine(const gp_graph *g, int32_t k, int64_t lmax, int32_t *part_inout, uint64_t seed,
                  int32_t global_iters, int32_t batch, int32_t queue, gp_mls_stats *st_host, void *ws,
                  size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || k > kMlsMaxK || lmax < 1 || global_iters < 0 || batch < 1 || batch > kMlsMaxBatch || queue < 1 ||
        queue > kMlsMaxQueue || !part_inout) {
        set_error("mls_refine: needs 1 <= k <= 256, lmax >= 1, global_iters >= 0, 1 <= batch <= 65536, "
                  "1 <= queue <= 64 and part");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    Timer t(stream);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    unsigned long long *bad = nullptr;
    GP_TRY(sc.alloc(&bad, 1));
    GP_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), stream));
    if (d.n > 0) {
        hipLaunchKernelGGL(k_check_blocks, dim3(grid_for(d.n, 256, 4096)), dim3(256), 0, stream, d.xadj, part_inout,
                           d.n, k, bad);
        GP_LAUNCH_CHECK();
    }
    unsigned long long hb = 0;
    GP_HIP(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, stream));
    GP_HIP(hipStreamSynchronize(stream));
    if (hb) {
        set_error("mls_refine: a vertex with neighbours has a block id outside [0, k)");
        return GP_ERR_GRAPH;
    }
    int64_t *B = nullptr;
    GP_TRY(sc.alloc(&B, k));
    GP_TRY(label_weights(d, part_inout, B, k, sc));
    MlsOut mo;
    GP_TRY(mls_refine(d, k, lmax, part_inout, B, nullptr, seed, global_iters, batch, queue, 50, 0.1, &mo, sc));
    const float ms = t.stop();
    if (st_host) {
        st_host->gain = mo.gain;
        st_host->searches = mo.searches;
        st_host->moves = mo.moves;
        st_host->local_iters = mo.local_iters;
        st_host->ms = ms;
        st_host->workspace_bytes = (int64_t)sc.high_water();
    }
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_contract(const gp_graph *g, const int32_t *labels, int32_t *xadj_c, int32_t *adjncy_c, int32_t *adjwgt_c,
                int32_t *vwgt_c, int32_t *f2c, int32_t *n_c_host, int32_t *nnz_c_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (!labels || !xadj_c || !vwgt_c || !f2c || (g->nnz > 0 && (!adjncy_c || !adjwgt_c))) {
        set_error("contract: an output or the labels array is NULL");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    unsigned long long *bad = nullptr;
    GP_TRY(sc.alloc(&bad, 1));
    GP_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), stream));
    if (d.n > 0) {
        hipLaunchKernelGGL(k_check_labels, dim3(grid_for(d.n, 256, 4096)), dim3(256), 0, stream, labels, d.n, d.n,
                           bad);
        GP_LAUNCH_CHECK();
    }
    unsigned long long hb = 0;
    GP_HIP(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, stream));
    GP_HIP(hipStreamSynchronize(stream));
    if (hb) {
        set_error("contract: a label is outside [0, n)");
        return GP_ERR_GRAPH;
    }
    CoarseOut co;
    co.xadj = xadj_c;
    co.adjncy = adjncy_c;
    co.adjwgt = adjwgt_c;
    co.vwgt = vwgt_c;
    co.f2c = f2c;
    GP_TRY(contract(d, labels, false, co, sc));
    if (n_c_host) *n_c_host = co.n;
    if (nnz_c_host) *nnz_c_host = co.nnz;
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_project(int32_t n, const int32_t *f2c, const int32_t *part_coarse, int32_t *part_fine, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!f2c || !part_coarse || !part_fine))) {
        set_error("project: n < 0 or an array is NULL");
        return GP_ERR_ARG;
    }
    GP_TRY(project(n, f2c, part_coarse, part_fine, stream));
    return GP_OK;
}

int gp_cut_and_blocks(const gp_graph *g, int32_t k, const int32_t *part, int64_t *cut_host, int64_t *block_w_dev,
                      void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || !part) {
        set_error("cut_and_blocks: k < 1 or part is NULL");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    int64_t *dcut = nullptr;
    GP_TRY(sc.alloc(&dcut, 1));
    GP_TRY(cut_dev(d, part, nullptr, dcut, sc));
    if (block_w_dev) GP_TRY(label_weights(d, part, block_w_dev, k, sc));
    if (cut_host) GP_HIP(hipMemcpyAsync(cut_host, dcut, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_partition(const gp_graph *g, int32_t k, double eps, const gp_params *p, int32_t *part_out,
                 gp_result *res_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || !(eps >= 0.0) || !part_out) {
        set_error("partition: k < 1, eps < 0 or part_out is NULL");
        return GP_ERR_ARG;
    }
    gp_params dp;
    gp_default_params(&dp);
    const gp_params *pp = p ? p : &dp;
    GP_TRY(check_params(pp, k, "partition"));
    return do_partition(g, k, eps, pp, part_out, res_host, ws, ws_bytes, stream);
}

int gp_coarsest(const gp_graph *g, int32_t k, double eps, const gp_params *p, int32_t *xadj_c, int32_t *adjncy_c,
                int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *part_c, int32_t *n_c_host, int32_t *nnz_c_host,
                void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || !(eps >= 0.0) || !xadj_c || !n_c_host || !nnz_c_host ||
        (g->n > 0 && (!vwgt_c || !part_c)) || (g->nnz > 0 && (!adjncy_c || !adjwgt_c))) {
        set_error("coarsest: k < 1, eps < 0 or an output is NULL");
        return GP_ERR_ARG;
    }
    gp_params dp;
    gp_default_params(&dp);
    const gp_params *pp = p ? p : &dp;
    GP_TRY(check_params(pp, k, "coarsest"));
    CoarsestOut co{xadj_c, adjncy_c, adjwgt_c, vwgt_c, part_c};
    GP_TRY(do_partition(g, k, eps, pp, nullptr, nullptr, ws, ws_bytes, stream, &co));
    *n_c_host = co.voff[1];
    *nnz_c_host = co.nnz;
    return GP_OK;
}

int gp_coarsest_batch(const gp_graph *g, int32_t G, const int32_t *vtx_off_host, const int32_t *k_host, double eps,
                      const gp_params *p, int32_t *xadj_c, int32_t *adjncy_c, int32_t *adjwgt_c, int32_t *vwgt_c,
                      int32_t *part_c, int32_t *vtx_off_c_host, int32_t *nnz_c_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (G < 1 || !vtx_off_host || !k_host || !(eps >= 0.0) || !xadj_c || !vtx_off_c_host || !nnz_c_host ||
        (g->n > 0 && (!vwgt_c || !part_c)) || (g->nnz > 0 && (!adjncy_c || !adjwgt_c))) {
        set_error("coarsest_batch: G < 1, eps < 0 or a required array is NULL");
        return GP_ERR_ARG;
    }
    GP_TRY(check_batch_layout(g, G, vtx_off_host, k_host, "coarsest_batch"));
    gp_params dp;
    gp_default_params(&dp);
    const gp_params *pp = p ? p : &dp;
    GP_TRY(check_params(pp, 1, "coarsest_batch"));
    if (pp->init_mode != GP_INIT_PLAIN) {
        set_error("coarsest_batch: the learned initial partition is available for single graphs only");
        return GP_ERR_ARG;
    }
    if (pp->active_set) {
        set_error("coarsest_batch: active-set rounds are available for single graphs only");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    CoarsestOut co{xadj_c, adjncy_c, adjwgt_c, vwgt_c, part_c};
    GP_TRY(partition_batch(d, G, vtx_off_host, k_host, eps, pp, nullptr, nullptr, sc, &co));
    for (int32_t q = 0; q <= G; q++) vtx_off_c_host[q] = co.voff[q];
    *nnz_c_host = co.nnz;
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int32_t gp_mpnn_param_count(int32_t k) { return k >= 1 && k <= kMpMaxK ? mpnn_param_count(k) : -1; }

int gp_mpnn_features(const gp_graph *g, uint64_t seed, float *X, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (g->n > 0 && !X) {
        set_error("mpnn_features: X is NULL");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    GP_TRY(mpnn_features(d, seed, false, X, nullptr, sc));
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_mpnn_forward(const gp_graph *g, int32_t k, const float *params, uint64_t seed, float *Z, int32_t *part,
                    void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || k > kMpMaxK || !params || (g->n > 0 && !Z && !part)) {
        set_error("mpnn_forward: k outside [1, 64], params NULL, or both outputs NULL");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    GP_TRY(mpnn_forward(d, k, params, seed, false, Z, part, nullptr, sc));
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_mpnn_decode(const gp_graph *g, int32_t k, const float *Z, int64_t lmax, int32_t *part, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || k > kMpMaxK || lmax < 1 || (g->n > 0 && (!Z || !part))) {
        set_error("mpnn_decode: k outside [1, 64], lmax < 1, or an array is NULL");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    GP_TRY(mpnn_decode(d, k, Z, lmax, false, part, sc));
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_mpnn_backward(const gp_graph *g, int32_t k, const float *params, uint64_t seed, const int32_t *target,
                     float lam, float *grad, double *loss_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (k < 1 || k > kMpMaxK || !params || !grad || (g->n > 0 && !target) || !(lam >= 0.0f)) {
        set_error("mpnn_backward: k outside [1, 64], lam < 0 or a required array is NULL");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    unsigned long long *bad = nullptr;
    GP_TRY(sc.alloc(&bad, 1));
    GP_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), stream));
    if (d.n > 0) {
        hipLaunchKernelGGL(k_check_labels, dim3(grid_for(d.n, 256, 4096)), dim3(256), 0, stream, target, d.n, k, bad);
        GP_LAUNCH_CHECK();
    }
    unsigned long long hb = 0;
    GP_HIP(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, stream));
    GP_HIP(hipStreamSynchronize(stream));
    if (hb) {
        set_error("mpnn_backward: a target block id is outside [0, k)");
        return GP_ERR_GRAPH;
    }
    GP_TRY(mpnn_backward(d, k, params, seed, target, lam, grad, loss_host, sc));
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return GP_OK;
}

int gp_mpnn_adam_step(float *params, float *m, float *v, const float *grad, int32_t count, int32_t step, float lr,
                      float beta1, float beta2, float eps, hipStream_t stream) {
    if (!params || !m || !v || !grad || count < 1 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
        set_error("mpnn_adam_step: NULL array, count < 1, step < 1 or a hyper-parameter out of range");
        return GP_ERR_ARG;
    }
    GP_TRY(mpnn_adam(params, m, v, grad, count, step, lr, beta1, beta2, eps, stream));
    return GP_OK;
}

int gp_partition_batch(const gp_graph *g, int32_t G, const int32_t *vtx_off_host, const int32_t *k_host, double eps,
                       const gp_params *p, int32_t *part_out, gp_result *res_host, void *ws, size_t ws_bytes, hipStream_t stream) {
    GP_TRY(check_ws(ws, ws_bytes));
    GP_TRY(check_graph_args(g));
    if (G < 1 || !vtx_off_host || !k_host || !(eps >= 0.0) || (g->n > 0 && !part_out)) {
        set_error("partition_batch: G < 1, eps < 0 or a required array is NULL");
        return GP_ERR_ARG;
    }
    GP_TRY(check_batch_layout(g, G, vtx_off_host, k_host, "partition_batch"));
    gp_params dp;
    gp_default_params(&dp);
    const gp_params *pp = p ? p : &dp;
    GP_TRY(check_params(pp, 1, "partition_batch"));
    if (pp->init_mode != GP_INIT_PLAIN) {
        set_error("partition_batch: the learned initial partition is available for single graphs only");
        return GP_ERR_ARG;
    }
    if (pp->active_set || pp->mls) {
        set_error("partition_batch: active-set rounds and the multi-try local search are available for single "
                  "graphs only");
        return GP_ERR_ARG;
    }
    Scratch sc(stream, ws, ws_bytes);
    const DevGraph d = dev_graph(g);
    GraphInfo gi;
    GP_TRY(graph_info(d, gi, sc));
    const int rc = partition_batch(d, G, vtx_off_host, k_host, eps, pp, part_out, res_host, sc, nullptr);
    if (rc >= 0 && res_host)
        for (int32_t q = 0; q < G; q++) res_host[q].workspace_bytes = (int64_t)sc.high_water();
    sc.release();
    GP_HIP(hipStreamSynchronize(stream));
    return rc;
}

const char *gp_strerror(int code) {
    switch (code) {
        case GP_OK: return "ok";
        case GP_WARN_IMBALANCED: return "partition is valid but a block exceeds L_max";
        case GP_ERR_ARG: return "invalid argument";
        case GP_ERR_GRAPH: return "invalid graph or labels";
        case GP_ERR_WORKSPACE: return "workspace too small";
        case GP_ERR_OVERFLOW: return "size or weight overflow";
        case GP_ERR_HIP: return "HIP runtime error";
        default: return "unknown error";
    }
}

const char *gp_last_error(void) { return gp::last_error(); }

void gp_profile_enable(int mode) {
    gp::prof_flush();
    gp::g_acc.clear();
    gp::g_ctx.clear();
    gp::g_prof = mode & (GP_PROFILE_KERNELS | GP_PROFILE_BY_LEVEL | GP_PROFILE_EAGER | GP_PROFILE_CALLS);
}

void gp_profile_select(const char *name) { gp::g_only = name ? name : ""; }

void gp_get_tuning(gp_tuning *t) {
    if (!t) return;
    const gp::Tuning &u = gp::tuning();
    for (int i = 0; i < 4; i++) t->tier_max[i] = u.tier_max[i];
    t->dense_split = u.dense_split;
    t->dense_chunk = u.dense_chunk;
}

int gp_set_tuning(const gp_tuning *t) {
    gp::Tuning u;
    if (t) {
        for (int i = 0; i < 4; i++) u.tier_max[i] = t->tier_max[i];
        u.dense_split = t->dense_split;
        u.dense_chunk = t->dense_chunk;
    }
    return gp::set_tuning(u);
}

int gp_release_cache(void) {
    std::lock_guard<std::mutex> lk(gp::g_arena_mu);
    int dev0 = 0;
    GP_HIP(hipGetDevice(&dev0));
    for (auto &kv : gp::g_arenas) {
        gp::Arena *a = kv.second;
        if (a->busy) {
            set_error("release_cache: a library call is still using the cache");
            return GP_ERR_ARG;
        }
    }
    for (auto &kv : gp::g_arenas) {
        GP_HIP(hipSetDevice(kv.first.first));
        GP_HIP(hipStreamSynchronize(kv.first.second));
        for (auto &b : kv.second->blocks) GP_HIP(hipFree(b.p));
        delete kv.second;
    }
    gp::g_arenas.clear();
    GP_HIP(hipSetDevice(dev0));
    return GP_OK;
}

int gp_profile_reserve(int launches) {
    gp::prof_flush();
    while ((int)gp::g_events.size() < 2 * launches) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return GP_ERR_HIP;
        gp::g_events.push_back(e);
    }
    return GP_OK;
}

int gp_profile_count(void) {
    gp::prof_flush();
    return (int)gp::g_acc.size();
}

int gp_profile_get(int i, char *name, int name_len, int64_t *launches, double *ms, double *bytes) {
    gp::prof_flush();
    if (i < 0 || i >= (int)gp::g_acc.size()) return GP_ERR_ARG;
    const auto &a = gp::g_acc[i];
    if (name && name_len > 0) {
        std::snprintf(name, (size_t)name_len, "%s", a.name.c_str());
    }
    if (launches) *launches = a.launches;
    if (ms) *ms = a.ms;
    if (bytes) *bytes = a.bytes;
    return GP_OK;
}

}  // extern "C"
