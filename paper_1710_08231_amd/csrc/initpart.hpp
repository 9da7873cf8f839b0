// initpart.hpp — initial partitioning and isolated-vertex placement (internal).
#pragma once
#include "lp.hpp"

namespace gp {

// Best of `attempts` tries (recursive BFS bisection -> LP refinement ->
// greedy rebalance) on g. part: [n] device output in [0, k) (-1 for vertices
// left out when skip_isolated is set). chosen_host (may be null) receives the
// index of the kept try.
int initial_partition(const DevGraph &g, bool skip_isolated, int32_t k, int64_t lmax, uint64_t seed,
                      int32_t attempts, int32_t rounds_refine, int32_t dir_alternate, bool wide, int32_t *part,
                      int32_t *chosen_host, Scratch &sc);

// Vertices without neighbours, in ascending id, each into the block that is
// lightest at that moment (ties -> lowest block id), starting from block
// weights B (device int64 [k], not modified).
int fill_isolated(const DevGraph &g, int32_t k, int32_t *part, const int64_t *B, int32_t *niso_host, Scratch &sc);

}  // namespace gp
