// contract.hpp — contraction, projection, cut (internal interface).
#pragma once
#include "lp.hpp"

namespace gp {

// rowof[e] = source vertex of directed entry e (inclusive max-scan of row starts).
int build_rowof(const DevGraph &g, int32_t *rowof, Scratch &sc);

struct CoarseOut {
    int32_t *xadj, *adjncy, *adjwgt, *vwgt, *f2c;  // device, sized for the fine graph
    int32_t n = 0, nnz = 0;                        // filled on return (host)
};

// Contraction of `labels` (values in [0, n)). When skip_isolated is set,
// vertices without neighbours are left out (f2c = -1) and no label of theirs
// is counted as used.
int contract(const DevGraph &g, const int32_t *labels, bool skip_isolated, CoarseOut &out, Scratch &sc);

// Upper bound of the scratch bytes contract() holds at once.
size_t contract_scratch_bound(int64_t n, int64_t nnz);

// part_fine[v] = f2c[v] >= 0 ? part_coarse[f2c[v]] : -1
int project(int32_t n, const int32_t *f2c, const int32_t *part_coarse, int32_t *part_fine, hipStream_t s);

// cut (device int64, each undirected edge once) of a partition; rowof may be null.
int cut_dev(const DevGraph &g, const int32_t *part, const int32_t *rowof, int64_t *cut_dev_out, Scratch &sc);

}  // namespace gp
