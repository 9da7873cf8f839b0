/*
 * oracle.h — plain, slow, single-threaded CPU oracle for size-constrained
 * label propagation (LP) clustering / refinement, contraction, projection,
 * initial partitioning and the multilevel driver.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it. It shares no code, header, table or
 * helper with the GPU library; the two only consume the same generated inputs.
 *
 * All arithmetic is integer: int32 weights, int64 sums. Every result is
 * therefore independent of summation order and must be matched bit-exactly.
 *
 * Readings of the paper used here (round-synchronous LP, direction
 * alternation, ascending-ID admission, stop rules, isolated-vertex handling,
 * the project-defined initial partitioner) are documented per function in
 * oracle.c.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;
    const int32_t *xadj;   /* [n+1] */
    const int32_t *adjncy; /* [xadj[n]] */
    const int32_t *adjwgt; /* [xadj[n]] or NULL = unit */
    const int32_t *vwgt;   /* [n] or NULL = unit */
} orc_graph;

typedef struct {
    int32_t rounds_run;
    int64_t moves;
    int64_t edge_visits;
} orc_lp_stats;

typedef struct {
    int32_t rounds_coarsen;   /* 10 */
    int32_t rounds_refine;    /* 25 */
    int32_t coarsest_per_k;   /* 60 */
    int32_t attempts;         /* 4 */
    int32_t stall_num;        /* 19 */
    int32_t stall_den;        /* 20 */
    int32_t dir_alternate;    /* 1 */
    uint64_t seed;
    int32_t init_mode;        /* 0 plain, 1 learned proposal judged against the plain one */
    int32_t mpnn_max_n;       /* learned proposal only when the coarsest graph has <= this many vertices */
    uint64_t mpnn_seed;       /* probe features */
    const float *mpnn_params; /* fp32 master weights (see orc_mpnn_param_count) */
    int32_t lp_async;         /* 0; 1: the paper's sequential LP, 2: colour-class LP, 3: colour-class
                                 LP in clustering only (oracle-only comparison modes) */
    int32_t active_set;       /* 0; bit 0: coarsening LP in active-set rounds, bit 1: uncoarsening LP */
    int32_t mls;              /* 0; g > 0: multi-try local search (g global iterations) after each level's
                                 LP refinement (oracle-only comparison mode) */
    int32_t init_fm;          /* 0; p > 0: at most p 2-way FM passes after every initial bisection */
    int32_t mls_batch;        /* 0: sequential MLS; b > 0: searches in batches of b (orc_mls_batched) */
    int32_t mls_queue;        /* 0: unbounded; q > 0: an MLS search queues at most q vertices */
} orc_params;

/* §III-C multi-try k-way local search (sequential, oracle-only; readings in mls.c) */
typedef struct {
    int64_t gain;        /* cut reduction */
    int64_t searches;    /* searches started */
    int64_t moves;       /* moves kept (best prefixes) */
    int64_t local_iters; /* local iterations over all global iterations */
} orc_mls_stats;
int64_t orc_mls(const orc_graph *g, int32_t k, int64_t lmax, int32_t *part, uint64_t seed, int32_t global_iters,
                double alpha, int32_t max_idle, orc_mls_stats *st);
/* The same with searches in batches of at most `batch` seeds (0: sequential), taken in
   queue order while the seeds' closed neighbourhoods are disjoint (the first seed
   whose neighbourhood meets a taken one starts the next batch): the searches of a
   batch start from the same partition and marks, and their kept prefixes are then
   applied in seed order with recomputed gains, each cut at its first move whose
   vertex has left its block or whose target is full, and kept up to its best
   recomputed prefix (§IV-C, ApplyMoves). batch = 1 gives the sequential result.
   max_queue > 0 bounds the vertices one search may queue (0: unbounded). */
int64_t orc_mls_batched(const orc_graph *g, int32_t k, int64_t lmax, int32_t *part, uint64_t seed,
                        int32_t global_iters, double alpha, int32_t max_idle, int32_t batch, int32_t max_queue,
                        orc_mls_stats *st);
/* gain of moving v to its best feasible adjacent block (*target, -1 if none) */
int64_t orc_mls_gain(const orc_graph *g, const int32_t *part, const int64_t *B, int32_t k, int64_t lmax, int32_t v,
                     int32_t *target);

/* LP flags (the former 0/1 direction argument is flag bit 0) */
#define ORC_LP_DIR_ALTERNATE 1
#define ORC_LP_ACTIVE_SET 2

typedef struct {
    int64_t cut, max_block_w, lmax, ucl;
    int32_t balanced, levels;
    int64_t edge_visits_cluster, edge_visits_refine;
    int32_t coarsest_n, n_isolated;
    int32_t learned_tried, learned_kept;
    int64_t plain_cut_coarsest, learned_cut_coarsest;
} orc_result;

/* Threads of the proposal loop of full LP rounds (default 1). Proposals are
 * pure functions of the round-start labels and weights, so every result is
 * the same for any thread count; only the time changes. */
void orc_set_threads(int32_t t);

int64_t orc_lmax(int64_t total_vwgt, int32_t k, double eps);
int64_t orc_total_vwgt(const orc_graph *g);

/* One LP round over all vertices; returns the number of admitted moves. */
int64_t orc_lp_round(const orc_graph *g, int32_t *C, int64_t *W, int32_t nlabels, int64_t U,
                     int32_t r, int32_t dir_alternate, int32_t *prop_out);

/* flags: ORC_LP_DIR_ALTERNATE | ORC_LP_ACTIVE_SET; edge_visits counts the
 * edges of the vertices evaluated (rounds_run * nnz without active sets) */
int orc_lp_cluster(const orc_graph *g, int64_t U, int32_t rounds, int32_t flags,
                   int32_t *labels_out, orc_lp_stats *st);
int orc_lp_refine(const orc_graph *g, int32_t k, int64_t lmax, int32_t rounds,
                  int32_t flags, int32_t *part_inout, orc_lp_stats *st);

/* §III-A sequential LP as the paper states it (queue by increasing degree,
 * in-place moves, neighbours of movers re-queued); an oracle-only mode. */
int orc_lp_cluster_async(const orc_graph *g, int64_t U, int32_t rounds, int32_t *labels_out, orc_lp_stats *st);
int orc_lp_refine_async(const orc_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t *part,
                        orc_lp_stats *st);

/* Colour-class LP, an oracle-only mode between the two above: the classes of a
 * first-fit colouring (decreasing splitmix64 priority) are visited one after
 * the other, each proposing from the current labels and admitting per target
 * in ascending id. orc_colour_classes writes colour[n] and returns the count. */
int32_t orc_colour_classes(const orc_graph *g, int32_t *colour);
int orc_lp_cluster_colour(const orc_graph *g, int64_t U, int32_t rounds, int32_t *labels_out, orc_lp_stats *st);
int orc_lp_refine_colour(const orc_graph *g, int32_t k, int64_t lmax, int32_t rounds, int32_t *part,
                         orc_lp_stats *st);

/* Coarse graph into caller buffers sized for the fine graph (n+1, nnz, nnz, n, n). */
int orc_contract(const orc_graph *g, const int32_t *labels, int32_t *xadj_c, int32_t *adjncy_c,
                 int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *f2c, int32_t *n_c, int32_t *nnz_c);

void orc_project(int32_t n, const int32_t *f2c, const int32_t *part_coarse, int32_t *part_fine);

int64_t orc_cut(const orc_graph *g, const int32_t *part);
void orc_block_weights(const orc_graph *g, const int32_t *part, int32_t k, int64_t *B);

uint64_t orc_mix4(uint64_t seed, uint64_t a, uint64_t base, uint64_t ks);

/* Recursive BFS-grow bisection of the whole graph (one attempt); fm_passes > 0
   runs at most that many 2-way FM passes after every bisection, a side that
   will hold j blocks weighing at most j * lmax (F4). */
void orc_recursive_bisection(const orc_graph *g, int32_t k, uint64_t seed, int32_t attempt, int64_t lmax,
                             int32_t fm_passes, int32_t *part_out);
/* Greedy rebalance; returns 1 if balanced afterwards, 0 if no move remained. */
int orc_rebalance(const orc_graph *g, int32_t k, int64_t lmax, int32_t *part);
/* Best of `attempts` (bisection -> lp_refine -> rebalance). Returns chosen attempt. */
int orc_initial_partition(const orc_graph *g, int32_t k, int64_t lmax, uint64_t seed,
                          int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, int32_t fm_passes,
                          int32_t *part_out);

/* Isolated-vertex fill; returns nothing, updates part and B. */
void orc_fill_isolated(const orc_graph *g, int32_t k, int32_t *part, int64_t *B);

int orc_partition(const orc_graph *g, int32_t k, double eps, const orc_params *p,
                  int32_t *part_out, orc_result *res);

/* Coarsest graph of the multilevel scheme (renumbered, without the vertices
 * that have no neighbour) and its initial partition, as orc_partition computes
 * them. Buffers sized as the input graph (n+1, nnz, nnz, n, n). */
int orc_coarsest(const orc_graph *g, int32_t k, double eps, const orc_params *p, int32_t *xadj_c,
                 int32_t *adjncy_c, int32_t *adjwgt_c, int32_t *vwgt_c, int32_t *part_c, int32_t *n_c,
                 int32_t *nnz_c);

/* Message-passing network for the learned initial partition (project addition;
 * it proposes the k-way assignment of the coarsest graph, §III-B's slot).
 * Features (18 per vertex): c(v)/c_max, deg(v)/max degree, 16 seeded +-1
 * probes smoothed by 8 lazy random-walk steps y <- (y + D^-1 A y) / 2.
 * Three layers h' = ReLU(b + Ws h + Wn m), m = (sum_u w(v,u) h_u) / sum_u w(v,u),
 * widths 18 -> 64 -> 64 -> 64, then z = bh + Wh h (k logits); block = argmax
 * (ties -> lowest). Weights are used rounded to bfloat16 (nearest-even);
 * sums are binary32 fused multiply-add chains in a fixed order (neighbours in
 * CSR order, inputs in index order). */
int32_t orc_mpnn_param_count(int32_t k);
float orc_bf16(float x);
void orc_mpnn_features(const orc_graph *g, uint64_t seed, float *X /* [n*18] */);
void orc_mpnn_infer(const orc_graph *g, int32_t k, const float *params, uint64_t seed, float *Z /* [n*k] */,
                    int32_t *part);
/* Capacity-respecting decoding of finite logits Z into blocks (see mpnn.c). */
void orc_mpnn_decode(const orc_graph *g, int32_t k, const float *Z, int64_t lmax, int32_t *part);

#ifdef __cplusplus
}
#endif
#endif
