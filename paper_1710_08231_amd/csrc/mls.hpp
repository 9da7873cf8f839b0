// mls.hpp — multi-try k-way local search after LP refinement (internal).
#pragma once
#include "lp.hpp"

namespace gp {

constexpr int kMlsMaxQueue = 64;   // largest per-search queue bound (one lane per queued vertex)
constexpr int kMlsMaxK = 256;      // largest block count
constexpr int kMlsMaxBatch = 65536;

struct MlsOut {
    int64_t gain = 0, searches = 0, moves = 0, local_iters = 0;
};

// Multi-try k-way local search (§III-C) in the batched form of §IV-C's
// parallel search: per global iteration the boundary vertices in a seeded
// hash order; per local iteration, batches of at most `batch` seeds whose
// closed neighbourhoods are pairwise disjoint run one search each from the
// batch's partition (each search queues at most `queue` vertices, moves by
// largest gain under lmax, stops after max_idle moves without a new best and
// keeps its shortest best prefix); the kept prefixes are then applied in seed
// order with recomputed gains, cut at a vertex that already left its block or
// a full target, and kept up to their best recomputed gain. part and B (the k
// block weights, device int64) are updated in place. hash_id (device, may be
// null = identity) gives the id each vertex has in the hash order (the rank
// among vertices with neighbours on an input graph). Labels < 0 take no part.
int mls_refine(const DevGraph &g, int32_t k, int64_t lmax, int32_t *part, int64_t *B, const int32_t *hash_id,
               uint64_t seed, int32_t global_iters, int32_t batch, int32_t queue, int32_t max_idle, double alpha,
               MlsOut *out, Scratch &sc);

}  // namespace gp
