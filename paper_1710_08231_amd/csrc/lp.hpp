// lp.hpp — host-side interface of the label-propagation rounds (internal).
#pragma once
#include <vector>

#include "gp_common.hpp"

namespace gp {

// Device view of a CSR graph (all pointers on the device).
struct DevGraph {
    int32_t n = 0, nnz = 0;
    const int32_t *xadj = nullptr, *adjncy = nullptr, *adjwgt = nullptr, *vwgt = nullptr;
};

// Per-call LP bookkeeping kept on the device so rounds need no host sync.
struct LPDev {
    int32_t round;  // index of the round the next launch sequence executes
    int32_t done;
    int32_t rounds_run;
    int32_t prev_moves;
    int32_t round_moves;
    int64_t total_moves;
    int64_t visits;  // active-set rounds: edges of the evaluated vertices
};

struct LPOut {
    int32_t rounds_run = 0;
    int64_t moves = 0;
    int64_t visits = 0;  // edge visits: rounds_run * nnz, or the active vertices' edges
    std::vector<int32_t> group_rounds;  // per group (when groups are given): its own rounds_run
    std::vector<int64_t> group_moves;
    // connection rows of a refinement run (all zero when every round gathered the labels)
    int64_t row_vertices = 0;  // vertices with a row
    int64_t row_entries = 0;   // their edges, gathered once to fill the rows
    int32_t row_width = 0;     // sums per row
    int32_t row_sum_bytes = 0;
    int64_t row_updates = 0;  // edges of the admitted movers pushed into rows
};

// Runs up to `rounds` synchronous LP rounds on (labels, W) in place.
//  labels [n]: current labels (-1 marks a vertex that takes no part: it
//              neither proposes nor counts toward W; such vertices must have
//              no neighbours).
//  W [nlabels]: label weights consistent with labels.
//  U: capacity of every label, or capv[L] per label when capv is given.
//  frozen (optional): vertices with frozen[v] != 0 keep their label and make
//  no proposal (their label weight still counts).
//  wide: use 64-bit connection sums.
// When `out` is non-null the stream is synchronised and statistics copied.
//  group/ngroups (optional): vertex groups (independent graphs of a batch);
//  out->group_rounds[q] then holds the rounds group q alone would have run
//  (two idle rounds in a row end a group; a group that went idle stays idle).
//  active: active-set rounds (§III-A/§IV-A queues, made synchronous): a
//  vertex is evaluated only while it owes evaluations; all start owing one
//  per direction (2 with dir_alternate, else 1), each evaluation pays one,
//  a proposal refused by capacity owes at least one more, and every
//  neighbour of an admitted mover owes one per direction again.
int lp_run(const DevGraph &g, int32_t *labels, int64_t *W, int32_t nlabels, int64_t U, int32_t rounds,
           int32_t dir_alternate, bool wide, LPOut *out, Scratch &sc, const int64_t *capv = nullptr,
           const uint8_t *frozen = nullptr, const int32_t *group = nullptr, int32_t ngroups = 0,
           bool active = false);

// Execution thresholds of the LP kernels. They choose which kernel serves a
// vertex and how big vertices are split; results never depend on them.
struct Tuning {
    int32_t tier_max[4] = {64, 256, 2048, 8192};  // hashed tables: degree bounds of the 32-lane,
                                                  // 64-lane, 256-thread and 512/1024-thread tiers
    int32_t dense_split = 256;                    // dense tables (k <= 256): rows above are chunked
    int32_t dense_chunk = 2048;                   // entries per chunk workgroup
};
Tuning &tuning();                  // process-wide, read at the start of every LP call
int set_tuning(const Tuning &t);   // validates against the table capacities

// Upper bound of the scratch bytes one lp_run over n vertices, nnz entries and
// nlabels labels holds at once, under the current tuning (either weight width).
size_t lp_scratch_bound(int64_t n, int64_t nnz, int64_t nlabels, bool active);

// Sum of edge weights (nnz if adjwgt is null); synchronises the stream.
int total_edge_weight(const DevGraph &g, int64_t *out, Scratch &sc);

// W[b] = sum of c(v) over v with labels[v] == b (labels < 0 skipped).
int label_weights(const DevGraph &g, const int32_t *labels, int64_t *W, int32_t nlabels, Scratch &sc);

}  // namespace gp
