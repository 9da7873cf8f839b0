// initpart.hpp — initial partitioning and isolated-vertex placement (internal).
#pragma once
#include <vector>

#include "lp.hpp"

namespace gp {

// G graphs side by side in one union graph: graph q owns vertices
// [voff[q], voff[q+1]) and blocks [kbase[q], kbase[q+1]) of k[q] blocks.
struct BatchInfo {
    int32_t G = 0;
    std::vector<int32_t> voff, k, kbase;  // host copies
    std::vector<int64_t> lmax;
    const int32_t *d_voff = nullptr, *d_kbase = nullptr, *d_gid = nullptr;  // device; gid[v] = graph of v
    const int64_t *d_lmax = nullptr;
};

// Outcome of an extra (learned) proposal per graph: the cuts (edge weight,
// each edge once) of the best plain try and of the proposal after the same
// refinement and rebalance, and whether the proposal was kept.
struct ProposalOut {
    std::vector<int64_t> plain_cut, prop_cut;
    std::vector<int32_t> kept;
};

// Best of `attempts` tries (recursive BFS bisection, each bisection followed
// by at most fm_passes 2-way FM passes -> LP refinement -> greedy rebalance)
// for every graph of the batch. part: [n] device output,
// global block ids kbase[q] + b (-1 for vertices left out when
// skip_isolated is set).
// extra (optional, device [n], graph-local block ids): one more proposal that
// goes through the same refinement and rebalance and is kept iff it is
// balanced and either the best plain try is not balanced or the proposal cuts
// no more edge weight (ties keep the proposal). `po` receives the outcome.
int initial_partition_batch(const DevGraph &g, bool skip_isolated, const BatchInfo &bi, uint64_t seed,
                            int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, int32_t fm_passes,
                            bool wide, int32_t *part, Scratch &sc, const int32_t *extra = nullptr,
                            ProposalOut *po = nullptr);

// The same for one graph (blocks [0, k)).
int initial_partition(const DevGraph &g, bool skip_isolated, int32_t k, int64_t lmax, uint64_t seed,
                      int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, int32_t fm_passes, bool wide,
                      int32_t *part, Scratch &sc, const int32_t *extra = nullptr, ProposalOut *po = nullptr);

// Batched placement of vertices without neighbours: per graph q, its
// isolated vertices (iso_first[q].. in the ascending list of all isolated
// vertices) go one by one to graph q's lightest block (global ids kbase[q]+b),
// starting from block weights B (device int64 [kbase[G]], not modified).
int fill_isolated_batch(const DevGraph &g, const BatchInfo &bi, const int32_t *d_iso_first, int32_t *part,
                        const int64_t *B, Scratch &sc);

// Caller buffers for the coarsest graph(s) and the initial partition (sized as
// the input graph). voff receives the per-graph vertex offsets (G+1), nnz the
// edge entries.
struct CoarsestOut {
    int32_t *xadj, *adjncy, *adjwgt, *vwgt, *part;
    std::vector<int32_t> voff;
    int32_t nnz = 0;
};

// Writes the top level gc (G graphs side by side, vertex offsets hvoff) with
// explicit weights and graph-local blocks. When level0 is set, gc is an input
// graph: its vertices without neighbours (niso[q] of graph q) are left out
// and the others renumbered in ascending order. P holds global block ids
// (kbase[gid[v]] + b; gid/d_kbase null for one graph).
int write_coarsest(const DevGraph &gc, bool level0, const int32_t *P, const int32_t *gid, const int32_t *d_kbase,
                   const std::vector<int32_t> &hvoff, const std::vector<int32_t> &niso, CoarsestOut &co,
                   Scratch &sc);

// gid[v] = q for v in [voff[q], voff[q+1]) (device arrays).
int graph_ids(int32_t G, int32_t n, const int32_t *d_voff, int32_t *gid, hipStream_t s);

// Vertices without neighbours, in ascending id, each into the block that is
// lightest at that moment (ties -> lowest block id), starting from block
// weights B (device int64 [k], not modified).
int fill_isolated(const DevGraph &g, int32_t k, int32_t *part, const int64_t *B, int32_t *niso_host, Scratch &sc);

}  // namespace gp
