// CPU check of the FMM tree (paper_1707_08369_amd/csrc/fmm_tree.h), built
// with g++ by tests/test_fmm_tree_cpu.py (under AddressSanitizer there).
//
// Reads cases from stdin: "K p" then K poles (ascending) and K roots. For
// each case it builds the tree and checks
//   1. every (target leaf, source leaf) pair of non-empty leaves is covered
//      exactly once: by the target's near list, or by one M2L pair of
//      ancestors (a pair with an empty leaf has nothing to evaluate);
//   2. every M2L pair is admissible: a positive gap at least the larger width;
//   3. every pole except the isolated one, and every root except the
//      directly evaluated ones, lies in its leaf's interval;
//   4. every directly evaluated root sees every non-empty leaf exactly once,
//      through one listed ancestor box (far field) or the leaf itself (exact);
//   5. list sizes fit the plan space the library reserves.
// Prints one line per case: "ok nlev near_max m2l_max opole outlier outlier2"
// or "FAIL <reason>".
#include <math.h>
#include <stdio.h>

#include <vector>

#include "../paper_1707_08369_amd/csrc/fmm_tree.h"

using namespace svdu;

static int check(int K, int p, const std::vector<double>& g, const std::vector<double>& mu) {
  FmmHostPlan P;
  fmm_build_tree(K, g.data(), mu.data(), p, &P);
  const int nlev = P.nlev, nleaf = 1 << nlev, leaf0 = fmm_box_id(nlev, 0);
  auto nonempty = [&](int id) { return P.s1[id] > P.s0[id]; };
  auto parent = [&](int id) { return (id - 1) / 2; };
  // 2. admissibility, and list sizes
  int m2l_max = 0, near_max = 0;
  for (int a = 0; a < P.nbox; ++a) {
    m2l_max = std::max(m2l_max, P.m2l_ptr[a + 1] - P.m2l_ptr[a]);
    near_max = std::max(near_max, P.near_ptr[a + 1] - P.near_ptr[a]);
    for (int q = P.m2l_ptr[a]; q < P.m2l_ptr[a + 1]; ++q) {
      const int b = P.m2l_src[q];
      if (b < 0 || b >= P.nbox) { printf("FAIL m2l source out of range\n"); return 1; }
      const double wa = P.hi[a] - P.lo[a], wb = P.hi[b] - P.lo[b];
      const double gap = std::max(P.lo[b] - P.hi[a], P.lo[a] - P.hi[b]);
      if (!(gap > 0.0 && gap >= std::max(wa, wb))) { printf("FAIL inadmissible m2l pair %d %d\n", a, b); return 1; }
    }
  }
  // the plan space of a product holds 2 * 64 list entries per box for the
  // M2L and near lists together, and nbox entries per directly evaluated
  // root for each of its two lists (a longer plan is refused with
  // SVDU_ENOMEM, never overrun)
  if (P.m2l_src.size() + P.near_src.size() > (size_t)128 * P.nbox ||
      P.dm2p.size() + P.dp2p.size() > (size_t)4 * P.nbox) {
    printf("FAIL lists exceed the reserved space\n");
    return 1;
  }
  // 1. exact coverage of leaf pairs
  std::vector<int> cover((size_t)nleaf * nleaf, 0);
  for (int a = 0; a < P.nbox; ++a) {
    int la = 0;
    while (fmm_box_id(la + 1, 0) <= a) ++la;
    for (int q = P.m2l_ptr[a]; q < P.m2l_ptr[a + 1]; ++q) {
      const int b = P.m2l_src[q];
      const int ka = a - fmm_box_id(la, 0), kb = b - fmm_box_id(la, 0);
      const int span = 1 << (nlev - la);
      for (int t = ka * span; t < (ka + 1) * span; ++t)
        for (int s = kb * span; s < (kb + 1) * span; ++s) cover[(size_t)t * nleaf + s] += 1;
    }
  }
  for (int t = 0; t < nleaf; ++t)
    for (int q = P.near_ptr[leaf0 + t]; q < P.near_ptr[leaf0 + t + 1]; ++q) {
      const int s = P.near_src[q] - leaf0;
      if (s < 0 || s >= nleaf) { printf("FAIL near source is not a leaf\n"); return 1; }
      cover[(size_t)t * nleaf + s] += 1;
    }
  for (int t = 0; t < nleaf; ++t)
    for (int s = 0; s < nleaf; ++s) {
      const bool need = nonempty(leaf0 + t) && nonempty(leaf0 + s);
      const int c = cover[(size_t)t * nleaf + s];
      if (need && c != 1) {   // pairs with an empty leaf evaluate nothing
        printf("FAIL leaf pair %d %d covered %d times\n", t, s, c);
        return 1;
      }
    }
  // 3. points in their leaves
  for (int i = 0; i < K; ++i) {
    const int id = leaf0 + i / P.s;
    if (i != P.opole && (g[i] < P.lo[id] || g[i] > P.hi[id])) { printf("FAIL pole %d outside its leaf\n", i); return 1; }
    if (i != P.outlier && i != P.outlier2 && (mu[i] < P.lo[id] || mu[i] > P.hi[id])) {
      printf("FAIL root %d outside its leaf\n", i);
      return 1;
    }
  }
  // 4. the directly evaluated roots
  int nd = 0;
  for (const int d : {P.outlier, P.outlier2}) {
    if (d < 0) continue;
    std::vector<int> seen(nleaf, 0);
    for (int q = P.dm2p_ptr[nd]; q < P.dm2p_ptr[nd + 1]; ++q) {
      const int b = P.dm2p[q];
      int lb = 0;
      while (fmm_box_id(lb + 1, 0) <= b) ++lb;
      const double gap = std::max(P.lo[b] - mu[d], mu[d] - P.hi[b]);
      if (!(gap > 0.0 && gap >= P.hi[b] - P.lo[b])) { printf("FAIL direct root far box too close\n"); return 1; }
      const int kb = b - fmm_box_id(lb, 0), span = 1 << (nlev - lb);
      for (int s = kb * span; s < (kb + 1) * span; ++s) seen[s] += 1;
    }
    for (int q = P.dp2p_ptr[nd]; q < P.dp2p_ptr[nd + 1]; ++q) seen[P.dp2p[q] - leaf0] += 1;
    for (int s = 0; s < nleaf; ++s)
      if (nonempty(leaf0 + s) && seen[s] != 1) {
        printf("FAIL direct root %d sees leaf %d %d times\n", d, s, seen[s]);
        return 1;
      }
    ++nd;
  }
  (void)parent;
  printf("ok %d %d %d %d %d %d\n", nlev, near_max, m2l_max, P.opole, P.outlier, P.outlier2);
  return 0;
}

int main() {
  int K = 0, p = 0, bad = 0;
  while (scanf("%d %d", &K, &p) == 2) {
    std::vector<double> g(K), mu(K);
    for (int i = 0; i < K; ++i)
      if (scanf("%lf", &g[i]) != 1) return 2;
    for (int i = 0; i < K; ++i)
      if (scanf("%lf", &mu[i]) != 1) return 2;
    bad |= check(K, p, g, mu);
    fflush(stdout);
  }
  return bad;
}
