/*
 * gp.h — C ABI of the MI355X (gfx950) size-constrained label-propagation
 * graph partitioner.
 *
 * Method: Akhremtsev, Sanders, Schulz, "High-Quality Shared-Memory Graph
 * Partitioning" (arXiv 1710.08231). The library implements the data-parallel
 * hot path of its multilevel scheme (§III, §IV): size-constrained label
 * propagation used to cluster (§III-A, §IV-A) and to refine a k-way partition
 * (§III-C, §IV-C with U = L_max), the contraction that builds each coarse
 * graph (§III-A, §IV-A), projection (§III-C), and a multilevel driver around
 * them with a project-defined initial partitioner (§III-B: recursive
 * bisection, best of several tries).
 *
 * Label propagation is round-synchronous: in round r every vertex proposes a
 * move from the labels and label weights of the round start; a move to label
 * L requires L != own label, (r even: L < own; r odd: L > own) when direction
 * alternation is on, W[L] + c(v) <= U (§II-A: a cluster is overloaded only
 * when it exceeds its bound), and a strictly larger connection than the own
 * label; ties go to the smallest label. The moves to one target t are
 * admitted in ascending vertex id while W[t] + (weight of all proposers to t
 * up to and including v) <= U (§IV-A: a move happens only if the cluster size
 * is still feasible). The call stops early after two idle rounds in a row.
 * Results are deterministic and bit-identical to the plain CPU definition.
 *
 * Conventions for every entry point
 *  - Graph: symmetric CSR, no self-loops, no duplicate edges, rows need not be
 *    sorted. All arrays inside gp_graph are DEVICE pointers on the current HIP
 *    device. adjwgt == NULL means unit edge weights, vwgt == NULL unit vertex
 *    weights. Weights are int32 >= 1; sums are int64.
 *  - Outputs named *_host are host pointers; every other array is a device
 *    pointer supplied and owned by the caller.
 *  - Work is ordered on `stream`. Calls that return host values synchronise
 *    the stream before returning.
 *  - Workspace. Every call that needs temporary device memory takes
 *    `void *ws, size_t ws_bytes` before the stream:
 *      ws != NULL: the call carves all its temporaries from the caller's
 *        device buffer [ws, ws + ws_bytes) (aligned up to 256 bytes first) and
 *        makes no device-memory allocation of its own. A buffer that turns
 *        out too small ends the call with GP_ERR_WORKSPACE (the outputs are
 *        then unspecified; gp_last_error() names the size reached). The
 *        buffer may be reused by the next call on the same stream at once.
 *        gp_workspace_bytes() gives a size that always suffices for the LP,
 *        contraction and cut calls; the multilevel calls need an amount that
 *        depends on the coarse graphs they build, reported afterwards in
 *        gp_result.workspace_bytes.
 *      ws == NULL (ws_bytes must be 0): the library takes the temporaries
 *        from a cache it keeps per (device, stream): blocks allocated
 *        stream-ordered (hipMallocAsync on `stream`) the first time a call
 *        needs them and reused by later calls; gp_release_cache() frees them.
 *    The library never frees caller memory. Concurrent calls on one stream
 *    from several host threads are not supported.
 *  - Return value: GP_OK (0), GP_WARN_IMBALANCED (1, valid result whose
 *    largest block exceeds L_max), or a negative error code; gp_strerror()
 *    and gp_last_error() describe it. On error the outputs are unspecified.
 *  - Global state: a thread-local last-error message; the process-wide LP
 *    execution thresholds (gp_set_tuning; they change speed, never results);
 *    the process-wide instrumentation switches (gp_profile_*); the
 *    per-(device, stream) scratch cache of ws == NULL calls; and a per-device
 *    static scratch array used only by gp_lp_refine_static. Calls with
 *    distinct outputs and distinct workspaces (or distinct streams) are
 *    independent.
 */
#ifndef GP_H
#define GP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GP_OK 0
#define GP_WARN_IMBALANCED 1
#define GP_ERR_ARG (-1)       /* NULL pointer, n < 0, k < 1, eps < 0, rounds < 0, U < 1 */
#define GP_ERR_GRAPH (-2)     /* bad offsets, neighbour id out of range, weight < 1, label out of range; with
                                 GP_VALIDATE=1 in the environment also a self-loop or an asymmetric graph */
#define GP_ERR_WORKSPACE (-3) /* the caller's workspace (or the static scratch) is too small */
#define GP_ERR_OVERFLOW (-4)  /* nnz >= 2^31 or a weight sum that does not fit its type */
#define GP_ERR_HIP (-5)       /* a HIP runtime call failed */

/* Initial partitioning of the coarsest graph (gp_params.init_mode). */
#define GP_INIT_PLAIN 0   /* best of `attempts` recursive bisections (§III-B) */
#define GP_INIT_LEARNED 1 /* plus the network's proposal, judged against them */

/* G = (V, E, c, w) of §II-A. n vertices, nnz = 2|E| directed CSR entries. */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *xadj;   /* [n+1], xadj[0] = 0, xadj[n] = nnz */
    const int32_t *adjncy; /* [nnz], neighbour ids in [0, n) */
    const int32_t *adjwgt; /* [nnz] edge weights w >= 1, or NULL for unit weights */
    const int32_t *vwgt;   /* [n] vertex weights c >= 1, or NULL for unit weights */
} gp_graph;

typedef struct {
    int32_t rounds_run;  /* rounds executed before the two-idle-rounds stop (<= rounds) */
    int64_t moves;       /* admitted moves summed over the rounds */
    int64_t edge_visits; /* rounds_run * nnz; with GP_LP_ACTIVE_SET the edges of the vertices evaluated */
    float ms;            /* device time of the call (HIP events on `stream`) */
    int64_t workspace_bytes; /* scratch the call held at once (see "Workspace" above) */
} gp_lp_stats;

/* Multilevel parameters; gp_default_params() fills the defaults shown. */
typedef struct {
    int32_t rounds_coarsen; /* 10: LP rounds per clustering (paper §VI configuration) */
    int32_t rounds_refine;  /* 25: LP rounds per refinement (paper §VI configuration) */
    int32_t coarsest_per_k; /* 60: coarsen while n > coarsest_per_k * k */
    int32_t attempts;       /* 4: initial partitioning tries (paper: max(p, 4)) */
    int32_t stall_num;      /* 19: stop after a level with stall_den*n' > stall_num*n */
    int32_t stall_den;      /* 20 */
    int32_t dir_alternate;  /* 1: direction alternation of synchronous rounds */
    uint64_t seed;          /* start-vertex hash of the initial bisections */
    int32_t init_mode;      /* GP_INIT_PLAIN; GP_INIT_LEARNED adds the network's proposal */
    int32_t mpnn_max_n;     /* 131072: the proposal is tried only on coarsest graphs this small (the
                               shipped k = 16 weights were trained on graphs of at most 3,252) */
    uint64_t mpnn_seed;     /* 0: seed of the network's probe features */
    const float *mpnn_params; /* NULL: device fp32 master weights, gp_mpnn_param_count(k) of them */
    int32_t active_set;     /* 0; bit 0: coarsening LP in active-set rounds (GP_LP_ACTIVE_SET), bit 1:
                               uncoarsening LP (3: both); single graphs only */
    int32_t init_fm;        /* 0; p > 0: after every bisection of the initial partitioning, at most p passes
                               of 2-way FM local search (§III-B: the bisection is improved by local search).
                               Only edges inside the bisected set count; a side that will hold j blocks may
                               weigh at most j * L_max; each pass keeps its shortest best prefix of moves
                               and stops after 50 moves without a new best; passes end early once one
                               gains nothing. Single graphs and batches. */
    int32_t mls;            /* 0; g > 0: after every level's LP refinement, multi-try k-way local search
                               (§III-C; gp_mls_refine) with g global iterations. Single graphs, k <= 256 */
    int32_t mls_batch;      /* 0: searches in batches of 1 (the sequential search); b > 0: batches of at most
                               b searches from one shared state (gp_mls_refine) */
    int32_t mls_queue;      /* 64: vertices one search may queue (1..64) */
} gp_params;

typedef struct {
    int64_t cut;          /* sum of w over edges between blocks, each edge once */
    int64_t max_block_w;  /* max_b c(V_b) */
    int64_t lmax;         /* (1+eps)*ceil(c(V)/k), floor of the binary64 product */
    int64_t ucl;          /* clustering bound max(c_max, lmax - ceil(c(V)/k)) */
    int32_t balanced;     /* max_block_w <= lmax */
    int32_t levels;       /* graphs in the hierarchy, level 0 included */
    int32_t coarsest_n;   /* vertices of the coarsest graph */
    int32_t n_isolated;   /* vertices without neighbours (placed at the end) */
    int64_t edge_visits_cluster; /* sum over levels of the clustering edge visits (gp_lp_stats) */
    int64_t edge_visits_refine;  /* same for refinement */
    float ms_coarsen, ms_init, ms_refine, ms_total; /* device-timed phases */
    int32_t learned_tried;        /* GP_INIT_LEARNED and the coarsest graph within mpnn_max_n */
    int32_t learned_kept;         /* the proposal replaced the plain initial partition */
    int64_t plain_cut_coarsest;   /* cut of the best plain try on the coarsest graph (-1: not tried) */
    int64_t learned_cut_coarsest; /* cut of the refined proposal (-1: not tried or discarded) */
    int64_t mls_gain;             /* cut reduction of the multi-try local search, summed over levels */
    int64_t workspace_bytes;      /* scratch the call held at once: a later call on the same graph with the
                                     same parameters and tuning succeeds with a workspace of this size
                                     (gp_partition_batch: the batch's, in every entry) */
} gp_result;

void gp_default_params(gp_params *p);

/*
 * Workspace size (bytes) that always suffices for one call of the kind `op`
 * on a graph of n vertices and nnz entries (k blocks for GP_OP_LP_REFINE; LP
 * flags as in the call), under the current execution thresholds
 * (gp_set_tuning). It is an upper bound assembled from the call's own
 * allocations at their largest sizes, so it is larger than what most graphs
 * need (gp_lp_stats.workspace_bytes reports what one call held). Returns 0
 * and sets the last error for invalid arguments or for a multilevel call,
 * whose need depends on the coarse graphs it builds: gp_partition and the
 * batched calls report theirs in gp_result.workspace_bytes. Host function.
 */
#define GP_OP_LP_CLUSTER 1
#define GP_OP_LP_REFINE 2
#define GP_OP_CONTRACT 3
#define GP_OP_CUT 4
size_t gp_workspace_bytes(int32_t op, int32_t n, int32_t nnz, int32_t k, int32_t flags);

/* §II-A balance bound: floor((1+eps) * ceil(total_vwgt / k)) in binary64. Pure host function. */
int64_t gp_lmax(int64_t total_vwgt, int32_t k, double eps);

/*
 * Flags of the LP calls (a plain 0/1 direction argument is flag bit 0).
 * GP_LP_DIR_ALTERNATE: even rounds consider only smaller labels, odd rounds
 * only larger ones. GP_LP_ACTIVE_SET: active-set rounds, the synchronous form
 * of the queues Q/Q' of §III-A and §IV-A. A vertex is evaluated (and its
 * edges visited) only while it owes evaluations. Every vertex starts owing
 * one per direction (2 with GP_LP_DIR_ALTERNATE, else 1). Each evaluation
 * pays one. A proposal refused by the admission leaves at least one owed.
 * Every neighbour of an admitted mover owes one per direction again. The
 * results differ from full rounds.
 */
#define GP_LP_DIR_ALTERNATE 1
#define GP_LP_ACTIVE_SET 2

/*
 * Size-constrained LP clustering (§III-A, §IV-A). Starts from singletons
 * (C[v] = v, W[v] = c(v)) and runs up to `rounds` rounds with bound U >= 1.
 * flags: GP_LP_DIR_ALTERNATE | GP_LP_ACTIVE_SET (other bits: GP_ERR_ARG).
 * labels_out: [n] device int32, receives cluster labels in [0, n) (leader ids,
 * not compacted). st_host (may be NULL) receives the statistics.
 */
int gp_lp_cluster(const gp_graph *g, int64_t U, int32_t rounds, int32_t flags,
                  int32_t *labels_out, gp_lp_stats *st_host, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * LP refinement (§III-C: LP started from a partition with U = L_max).
 * part_inout: [n] device int32 with 0 <= part[v] < k; overwritten with the
 * refined partition. lmax >= 1 bounds every block.
 * With ws == NULL on graphs above 16,384 vertices, the block connections of
 * every vertex above KT/8 neighbours (KT = k rounded up to 16, 64 or 256)
 * are kept from round to round in the cache (KT sums per such vertex) and
 * changed only by the admitted moves; this takes the edge weights of u's list
 * for both (u, v) and (v, u), as in any graph of §II-A. The result equals the
 * plain rounds', which a caller workspace and GP_REFINE_ROWS=0 select.
 */
int gp_lp_refine(const gp_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t flags,
                 int32_t *part_inout, gp_lp_stats *st_host, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * gp_lp_refine for callers that cannot allocate device memory: code that runs
 * under HIP graph capture, tight serving loops, and harnesses that forbid
 * allocation. Same arguments (without a workspace) and same results as
 * gp_lp_refine, but the temporaries come from a static scratch array of 64
 * MiB that the library holds on every GPU it runs on until the process ends,
 * and the call creates no HIP events, streams or graphs (every round is
 * launched directly; st_host->ms is the host time of the call). Sizes whose
 * gp_workspace_bytes(GP_OP_LP_REFINE, n, nnz, k, flags) exceeds 64 MiB are
 * rejected with GP_ERR_WORKSPACE before any device work (about n <= 700,000
 * with 16 entries per vertex and k <= 64 under the default thresholds). All
 * calls on one GPU share that GPU's array: calls that overlap on one GPU
 * (several streams or host threads) race and must not be issued.
 */
int gp_lp_refine_static(const gp_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t flags,
                        int32_t *part_inout, gp_lp_stats *st_host, hipStream_t stream);

/*
 * Multi-try k-way local search (§III-C) on a k-way partition, in the batched
 * form of §IV-C's parallel search (PerformMoves on every PE, then ApplyMoves):
 *  - a global iteration visits the boundary vertices in a seeded hash order
 *    (key splitmix64(h ^ v), h chained from seed, global and local iteration);
 *  - a local iteration takes them in batches: the next at most `batch` seeds
 *    not marked at the batch's start, ending before the first one whose
 *    closed neighbourhood meets an earlier seed's;
 *  - every seed of a batch starts one search from the batch's partition and
 *    marks (one wavefront each, none sees the others' moves): it queues the
 *    seed and its unmarked neighbours, at most `queue` vertices in all;
 *    repeatedly takes the queued vertex of largest gain (ties: lower id),
 *    re-queues it if its gain changed, else moves it to its best block (the
 *    largest connection to an adjacent other block with room under lmax,
 *    ties: lowest block; gain = that connection minus the one to its own
 *    block); re-evaluates queued neighbours and queues unmarked ones; stops on
 *    an empty queue or after 50 moves without a new best; keeps its shortest
 *    prefix of largest positive cumulative gain;
 *  - the kept prefixes are applied in seed order with gains recomputed on the
 *    current partition (ApplyMoves), each cut at a vertex that already left
 *    its block or a target without room and kept up to its best recomputed
 *    gain, so lmax is never broken; the searches' queued vertices stay marked
 *    for the rest of the local iteration;
 *  - the vertices moved in a local iteration are the next one's todo list
 *    while its gain exceeds 10% of the global iteration's gain so far.
 * part_inout: [n] device int32 in [0, k) (vertices without neighbours may hold
 * -1), overwritten. 1 <= k <= 256, 1 <= queue <= 64, 1 <= batch <= 65536.
 * st_host (may be NULL): gain (cut reduction), searches, kept moves, local
 * iterations. Results are deterministic.
 */
typedef struct {
    int64_t gain, searches, moves, local_iters;
    float ms;
    int64_t workspace_bytes;
} gp_mls_stats;
int gp_mls_refine(const gp_graph *g, int32_t k, int64_t lmax, int32_t *part_inout, uint64_t seed,
                  int32_t global_iters, int32_t batch, int32_t queue, gp_mls_stats *st_host, void *ws,
                  size_t ws_bytes, hipStream_t stream);

/*
 * Contraction (§III-A; coarse ids by a prefix sum over used labels, §IV-A).
 * labels: [n] device int32 in [0, n). Coarse vertex i = the rank of its label
 * among the used labels; c'(i) = sum of c over the cluster; the coarse edge
 * (i, j), i != j, carries the summed weight of fine edges between the two
 * clusters. Coarse rows ascending, columns ascending within a row.
 * Outputs (device, caller-sized for the fine graph): xadj_c [n+1],
 * adjncy_c [nnz], adjwgt_c [nnz], vwgt_c [n], f2c [n] (fine -> coarse id).
 * n_c_host / nnz_c_host receive the coarse sizes.
 */
int gp_contract(const gp_graph *g, const int32_t *labels, int32_t *xadj_c, int32_t *adjncy_c,
                int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *f2c, int32_t *n_c_host,
                int32_t *nnz_c_host, void *ws, size_t ws_bytes, hipStream_t stream);

/* Projection (§III-C): part_fine[v] = part_coarse[f2c[v]] for v < n (device arrays). */
int gp_project(int32_t n, const int32_t *f2c, const int32_t *part_coarse, int32_t *part_fine,
               hipStream_t stream);

/* §II-A cut (each undirected edge once) and block weights B[k] (device int64) of a partition. */
int gp_cut_and_blocks(const gp_graph *g, int32_t k, const int32_t *part, int64_t *cut_host,
                      int64_t *block_w_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Multilevel k-way partition (§III scheme): coarsen with gp_lp_cluster /
 * gp_contract under U = max(c_max, L_max - ceil(c(V)/k)) while
 * n > coarsest_per_k * k (vertices without neighbours are set aside first;
 * a level that does not shrink is discarded; a level with
 * stall_den * n' > stall_num * n is the last), partition the coarsest graph
 * (best of `attempts` recursive BFS bisections, each followed by LP
 * refinement and a greedy rebalance), then project and refine every level
 * with U = L_max, and place vertices without neighbours, in ascending id,
 * into the currently lightest block.
 * With init_mode = GP_INIT_LEARNED (a project addition in the slot of §III-B)
 * and a coarsest graph of at most mpnn_max_n vertices, the network of
 * gp_mpnn_forward also proposes an assignment of the coarsest graph (its
 * logits decoded by gp_mpnn_decode with L_max); the proposal goes through the
 * same LP refinement and rebalance as
 * every bisection try and replaces the best plain try iff it is balanced and
 * either the plain try is not or it cuts no more edge weight (ties keep the
 * proposal). A proposal with a NaN or infinite logit is discarded. Requires
 * k <= 64 and mpnn_params.
 * 1 <= k <= 2048: the initial partitioner's rebalance keeps per-block state
 * in LDS; a larger k returns GP_ERR_ARG once the coarsest graph is reached.
 * part_out: [n] device int32 in [0, k). res_host may be NULL.
 * Returns GP_OK, GP_WARN_IMBALANCED, or an error.
 */
int gp_partition(const gp_graph *g, int32_t k, double eps, const gp_params *p, int32_t *part_out,
                 gp_result *res_host, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * The coarsest graph of gp_partition's hierarchy and its initial partition
 * (the pairs the learned proposal is trained on). Vertices without
 * neighbours are left out and the others renumbered in ascending order when
 * no coarsening happened. Outputs (device, sized as the input graph): xadj_c
 * [n+1], adjncy_c [nnz], adjwgt_c [nnz], vwgt_c [n], part_c [n] in [0, k);
 * n_c_host / nnz_c_host receive the sizes.
 */
int gp_coarsest(const gp_graph *g, int32_t k, double eps, const gp_params *p, int32_t *xadj_c, int32_t *adjncy_c,
                int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *part_c, int32_t *n_c_host, int32_t *nnz_c_host,
                void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * gp_coarsest for the G graphs of a disjoint-union graph at once (layout as in
 * gp_partition_batch), through the batched form. The coarsest graphs are
 * written side by side: graph q owns coarse vertices [vtx_off_c_host[q],
 * vtx_off_c_host[q+1]) (G+1 host entries) and only edges among them;
 * part_c holds graph-local block ids. Every graph's result equals gp_coarsest
 * on that graph alone.
 */
int gp_coarsest_batch(const gp_graph *g, int32_t G, const int32_t *vtx_off_host, const int32_t *k_host, double eps,
                      const gp_params *p, int32_t *xadj_c, int32_t *adjncy_c, int32_t *adjwgt_c, int32_t *vwgt_c,
                      int32_t *part_c, int32_t *vtx_off_c_host, int32_t *nnz_c_host, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * The learned initial partition's network (a project addition; it fills the
 * slot of §III-B's initial partitioning). Per vertex v:
 *   features  X[v] = (c(v)/c_max, deg(v)/max deg, y_8[v][0..15]); y_0 = 16
 *             seeded +-1 probes (splitmix64 of splitmix64(seed) ^ (16 v + j),
 *             sign from the top bit), y_{t+1}[v] = (y_t[v] + sum_u w(v,u) y_t[u] / d(v)) / 2
 *             with d(v) the weighted degree (a vertex without neighbours keeps y);
 *   layers    h_l = ReLU(b_l + Ws_l h_{l-1}[v] + Wn_l m_l[v]), m_l[v] = sum_u w(v,u) h_{l-1}[u] / d(v)
 *             (0 without neighbours), widths 18 -> 64 -> 64 -> 64;
 *   head      z[v] = bh + Wh h_3[v] (k logits), block = argmax, ties -> lowest.
 * Parameters (fp32 master weights, flat, device): per layer Ws [64][d_in],
 * Wn [64][d_in], b [64]; then Wh [k][64], bh [k]; row-major, output index
 * first. gp_mpnn_param_count(k) of them (19,920 for k = 16), 1 <= k <= 64
 * (returns -1 otherwise). The forward pass uses them rounded to bfloat16
 * (nearest, ties to even) and is bit-reproducible: sums are binary32 fused
 * multiply-add chains in a fixed order (neighbours in CSR order, inputs in
 * index order after the bias, self before aggregated inputs); 1/d(v) and the
 * two ratio features are binary64 divisions rounded once.
 */
int32_t gp_mpnn_param_count(int32_t k);

/* Features X: [n*18] device float (row-major per vertex). */
int gp_mpnn_features(const gp_graph *g, uint64_t seed, float *X, void *ws, size_t ws_bytes, hipStream_t stream);

/* Logits Z [n*k] and argmax blocks part [n] (device; either may be NULL). */
int gp_mpnn_forward(const gp_graph *g, int32_t k, const float *params, uint64_t seed, float *Z, int32_t *part,
                    void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Capacity-respecting decoding of finite logits Z [n*k] (device) into blocks
 * part [n] (device), under the block bound lmax (the admission rule of an LP
 * move, §IV-A): every vertex ranks the blocks by logit, highest first (ties
 * -> lower block); in round r = 0..k-1 every vertex not yet placed offers its
 * r-th block, and the offers to block t are admitted in ascending vertex id
 * while B[t] + (weight of all offers to t up to and including v) <= lmax;
 * vertices still unplaced after k rounds go, in ascending id, to the block
 * that is lightest at that moment (ties -> lower block). 1 <= k <= 64.
 */
int gp_mpnn_decode(const gp_graph *g, int32_t k, const float *Z, int64_t lmax, int32_t *part, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Training loss and gradient (binary32, within tolerance of the exact
 * gradient). With S = softmax(z) per vertex, target t [n] in [0, k) (device):
 *   edge  = (1/Omega) sum over directed CSR entries (v,u) of w(v,u) BCE(p, [t_v == t_u]),
 *           p = <S_v, S_u> clipped to [1e-6, 1 - 1e-6] (zero gradient outside),
 *           Omega = sum of all entries of adjwgt;
 *   bal   = lam * k * sum_c (Q_c - 1/k)^2, Q_c = sum_v c(v) S_v[c] / c(V).
 * grad: [P] device float, overwritten with d(edge + bal)/d(weights) taken at
 * the bfloat16-rounded weights. loss_host (may be NULL): {edge, bal}.
 */
int gp_mpnn_backward(const gp_graph *g, int32_t k, const float *params, uint64_t seed, const int32_t *target,
                     float lam, float *grad, double *loss_host, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adam on the master weights (device arrays of `count` floats): m = b1 m +
 * (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * step >= 1 counts the updates made so far including this one.
 */
int gp_mpnn_adam_step(float *params, float *m, float *v, const float *grad, int32_t count, int32_t step, float lr,
                      float beta1, float beta2, float eps, hipStream_t stream);

/*
 * Batched form (a project addition; §III scheme per graph): G independent
 * graphs stored side by side as one disjoint-union graph g — graph q owns
 * vertices [vtx_off_host[q], vtx_off_host[q+1]) and no edge joins two graphs
 * (GP_ERR_GRAPH otherwise). Graph q is cut into k_host[q] blocks with the
 * balance bound of its own total weight. All graphs are coarsened and refined
 * together level by level through the same kernels (per-label capacities,
 * graphs that stopped coarsening are carried along unchanged), and one
 * batched initial partitioning runs on the coarsest level. The result for
 * every graph equals gp_partition on that graph alone (same parameters).
 * part_out: [n] device int32, block ids local to each graph (0 <= b < k[q]),
 * 1 <= k[q] <= 2048 as in gp_partition.
 * res_host: [G] host results (may be NULL); the ms_* fields are batch totals.
 * Returns GP_OK, GP_WARN_IMBALANCED (some graph imbalanced), or an error.
 */
int gp_partition_batch(const gp_graph *g, int32_t G, const int32_t *vtx_off_host, const int32_t *k_host, double eps,
                       const gp_params *p, int32_t *part_out, gp_result *res_host, void *ws, size_t ws_bytes, hipStream_t stream);

const char *gp_strerror(int code);
const char *gp_last_error(void);

/*
 * Execution thresholds of the LP kernels (process-wide; results never depend
 * on them, only speed). tier_max: upper degree bounds of the hashed-table
 * tiers served by 32 lanes, 64 lanes, one workgroup (128 threads up to
 * degree 1024, 256 threads above) and a larger workgroup (512 threads up to
 * degree 4096, 1024 threads above) (defaults 64,
 * 256, 2048, 8192 — also the largest allowed, as each tier's table holds
 * twice its bound; non-decreasing, tier_max[0] >= 16);
 * vertices above the last bound take the multi-workgroup path. dense_split:
 * with k <= 256 labels, rows above this degree are split into chunks of
 * dense_chunk entries, one workgroup each (defaults 256 and 2048).
 * gp_set_tuning(NULL) restores the defaults; invalid values give GP_ERR_ARG.
 * Chosen per workload by paper_1710_08231_amd/autotune.py.
 */
typedef struct {
    int32_t tier_max[4];
    int32_t dense_split;
    int32_t dense_chunk;
} gp_tuning;
void gp_get_tuning(gp_tuning *t);
int gp_set_tuning(const gp_tuning *t);

/* Frees the library's cached device memory of every (device, stream) after
 * synchronising those streams. Must not run while a library call is active. */
int gp_release_cache(void);

/*
 * Instrumentation for measurement (not part of the method). Per entry name
 * the library accumulates the number of recorded launches, their summed
 * device time (ms, HIP events on the caller's stream) and their summed
 * algorithmic bytes (CSR, weight and label bytes the work must move; see the
 * kernel sources). gp_profile_enable(mode) clears the counters and starts
 * recording with the mode bits below; gp_profile_enable(0) stops.
 *   GP_PROFILE_KERNELS  every launch of an LP proposal kernel is bracketed;
 *                       rounds are then launched one by one (no replay).
 *   GP_PROFILE_EAGER    only the proposal launches of the first round of
 *                       every LP run; the later rounds run without events, so
 *                       the timed path stays the production one.
 *   GP_PROFILE_CALLS    every LP run inside gp_partition is bracketed and
 *                       recorded as "lp_cluster" or "lp_refine", with the
 *                       run's algorithmic bytes: per edge visit the neighbour
 *                       id, its weight when present and its label (4 bytes
 *                       clustering, 1 refining), per vertex and round 12
 *                       bytes (+4 with vertex weights), per admitted move 16;
 *                       and every contraction, as "contract", with its
 *                       algorithmic bytes: the fine graph read once (row
 *                       offsets, labels, neighbour ids, weights), one coarse
 *                       id gathered per entry, f2c and the coarse graph
 *                       written.
 *   GP_PROFILE_BY_LEVEL names entries "cluster L<l>|<kernel>",
 *                       "refine L<l>|<kernel>", "contract L<l>|contract" or
 *                       "init|<kernel>".
 * gp_profile_get copies entry i (0 <= i < gp_profile_count()) into caller
 * memory; name is NUL-terminated and truncated to name_len bytes. Host-only,
 * not thread safe.
 */
#define GP_PROFILE_KERNELS 1
#define GP_PROFILE_BY_LEVEL 2
#define GP_PROFILE_EAGER 4
#define GP_PROFILE_CALLS 8
void gp_profile_enable(int mode);
/* Restrict recording to launches of kernel `name` (NULL: record all). */
void gp_profile_select(const char *name);
/* Create the HIP events for `launches` recorded launches ahead of time, so
 * that recording inside a timed region creates none. */
int gp_profile_reserve(int launches);
int gp_profile_count(void);
int gp_profile_get(int i, char *name, int name_len, int64_t *launches, double *ms, double *bytes);

#ifdef __cplusplus
}
#endif
#endif
