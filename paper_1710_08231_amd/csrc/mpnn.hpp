// mpnn.hpp — the message-passing network that proposes the initial k-way
// assignment of the coarsest graph (internal interface).
#pragma once
#include "lp.hpp"

namespace gp {

constexpr int kMpProbe = 16;               // seeded +-1 probe vectors
constexpr int kMpWalk = 8;                 // lazy random-walk smoothing steps
constexpr int kMpFeat = 2 + kMpProbe;      // c/c_max, deg/max_deg, probes
constexpr int kMpHid = 64;                 // hidden width of the three layers
constexpr int kMpMaxK = 64;                // head width limit (one wavefront per vertex)

int32_t mpnn_param_count(int32_t k);

// Features X [n][18] (device). active_only: vertices without neighbours are
// left out of c_max and the probe stream is indexed by each other vertex's
// rank among them (the graph of a level whose isolated vertices were set
// aside). rinv (device [n], optional) receives 1/sum of edge weights.
int mpnn_features(const DevGraph &g, uint64_t seed, bool active_only, float *X, float *rinv, Scratch &sc);

// Logits Z [n][k] and argmax blocks part [n] (either may be null) with the
// master weights `params` (device fp32) rounded to bfloat16. nonfinite_dev
// (optional, device int32, zeroed by the caller) is set to 1 when a logit of a
// taking-part vertex is NaN or infinite.
int mpnn_forward(const DevGraph &g, int32_t k, const float *params, uint64_t seed, bool active_only, float *Z,
                 int32_t *part, int32_t *nonfinite_dev, Scratch &sc);

// Capacity-respecting decoding of finite logits Z [n][k] into blocks part [n]
// (vertices ranked by logit per block; round r admits each unplaced vertex's
// r-th block in ascending id while the block stays within lmax; leftovers to
// the lightest block). active_only: vertices without neighbours take no part.
int mpnn_decode(const DevGraph &g, int32_t k, const float *Z, int64_t lmax, bool active_only, int32_t *part,
                Scratch &sc);

// Training loss (edge term, balance term) and its gradient w.r.t. the master
// weights (straight through the bfloat16 rounding), grad: device [P].
int mpnn_backward(const DevGraph &g, int32_t k, const float *params, uint64_t seed, const int32_t *target,
                  float lam, float *grad, double *loss_host, Scratch &sc);

// One Adam step on the master weights (bias-corrected moments m, v).
int mpnn_adam(float *params, float *m, float *v, const float *grad, int32_t count, int32_t step, float lr, float b1,
              float b2, float eps, hipStream_t s);

}  // namespace gp
