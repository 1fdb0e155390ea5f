// Host-side plan of one FMM product (see k_fmm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "fmm_tree.h"
#include "svdu_internal.h"

namespace svdu {

struct FmmPrepared {
  FmmHostPlan P;
  size_t off[11];
};

// Builds the plan of one product from host copies of the stage's K poles g
// (ascending) and roots mu, and appends its arrays to `blob`.
void fmm_prepare(int K, const double* g_host, const double* mu_host, double eps, std::vector<char>* blob,
                 FmmPrepared* out);
// Enqueues X_out = X C~ (times colscale per output column, if given) for
// stage s with a plan whose blob was uploaded to plan_dev. 0, or -2 when the
// work area is too small.
int fmm_launch(int R, const double* X, int ldx, const Stage& s, const FmmPrepared& pp, const char* plan_dev,
               double* Xo, int ldo, const double* colscale, double* work, size_t work_elems, hipStream_t st);

}  // namespace svdu
