// Many small, uneven SDPs in one persistent launch (batched.hip).
#pragma once

#include "../../include/wcsdp.h"
#include "common.hpp"

namespace wc {

using BatchTune = sdp_batch_tune;

// Solve `count` problems (dense constraint matrices only) with one persistent
// kernel; results[i] receives the statistics, X_out[i] (device, n_i x n_i)
// the primal solution when X_out and X_out[i] are non-null.  `tune` holds one
// configuration per instance (null: defaults).
void solve_batched(const sdp_problem* probs, int count, const sdp_options* opt, hipStream_t st, sdp_result* results,
                   double* const* X_out, double* const* y_out, const BatchTune* tune);

// Autotuner: times each candidate configuration on a sample of the instances
// of every size bucket (n < 48, n < 96, larger) for a fixed number of
// interior-point iterations and returns the fastest per instance.
void autotune_batched(const sdp_problem* probs, int count, const sdp_options* opt, hipStream_t st, BatchTune* out,
                      double* bucket_ms);

}  // namespace wc
