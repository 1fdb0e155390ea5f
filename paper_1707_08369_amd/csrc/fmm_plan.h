// Host-side plan of one FMM product (see k_fmm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "svdu_internal.h"

namespace svdu {

struct FmmHostPlan {
  int p = 0, s = 0, K = 0, nlev = 0, nbox = 0;
  int outlier = -1;                 // root outside [g_0, g_K-1], evaluated directly
  int outlier2 = -1;                // root in the gap next to an isolated pole, evaluated directly
  int opole = -1;                   // isolated extreme pole: in no box interval, applied to every root directly
  std::vector<double> lo, hi;       // box intervals
  std::vector<int> s0, s1;          // source / target index range of each box
  std::vector<int> m2l_ptr, m2l_src;
  std::vector<int> near_ptr, near_src;
  std::vector<int> lev_off;         // first box id of each level
  // the directly evaluated roots (outlier, then outlier2, those that exist):
  // boxes whose expansion converges at the root, and leaves summed exactly
  std::vector<int> dm2p, dp2p;
  int dm2p_ptr[3] = {0, 0, 0}, dp2p_ptr[3] = {0, 0, 0};
};

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
