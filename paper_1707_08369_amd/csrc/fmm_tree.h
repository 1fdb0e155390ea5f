// Host-side tree of the row-batched 1-D FMM (Section 5 and Appendix D of the
// paper): box intervals, the M2L and near-field lists of a dual traversal, and
// the lists of the directly evaluated roots. Plain C++ (no HIP), so that the
// tree can be built and checked on a CPU alone.
#pragma once
#include <math.h>

#include <algorithm>
#include <utility>
#include <vector>

namespace svdu {

// Largest expansion order the kernels hold (padded length of a coefficient
// vector).
constexpr int kFmmMaxOrder = 16;

// Box k of level l in the array of a full binary tree.
constexpr int fmm_box_id(int l, int k) { return (1 << l) - 1 + k; }

// p = ceil(log_5(1/eps)) for 0 < eps < 1 (Appendix D Step 1, read with
// 0 < eps < 1): the order whose interpolation error (3 + sqrt 8)^-p, about
// 5^-p, meets eps.
inline int fmm_required_order(double eps) { return (int)ceil(log(1.0 / eps) / log(5.0)); }

// The order the kernels run: the required order, at least 8 (leaves of 16 to
// 32 poles). Callers reject an eps whose required order exceeds kFmmMaxOrder.
inline int fmm_order(double eps) { return std::min(kFmmMaxOrder, std::max(8, fmm_required_order(eps))); }

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

// Builds the tree of one product over K poles g (ascending) and K roots mu
// (root i interlaces into the interval of pole i) for expansion order p.
inline void fmm_build_tree(int K, const double* g, const double* mu, int p, FmmHostPlan* P) {
  P->p = p;
  P->K = K;
  // a full binary tree whose leaves hold at most 32 poles each
  int nlev = 0;
  while ((K + (1 << nlev) - 1) >> nlev > 32) ++nlev;
  P->s = (K + (1 << nlev) - 1) >> nlev;
  const int s = P->s;
  // The extreme root (beyond the last pole for rho > 0, before the first for
  // rho < 0) can lie far outside the spectrum; it is kept out of the box
  // intervals, which would otherwise make its leaf, and every box above it,
  // inadmissible to all, and is evaluated on its own (fmm_direct_roots).
  P->outlier = -1;
  for (int i = 0; i < K; ++i)
    if (mu[i] > g[K - 1] || mu[i] < g[0]) P->outlier = i;
  // An extreme pole far from the others (the previous level's extreme root
  // becomes one) would stretch its leaf across the whole gap and leave it
  // near to almost every leaf; such a pole stays out of the box intervals,
  // the multipole expansions and the near fields, and its charge is applied
  // to every root directly. The root that interlaces into that gap, when it
  // lies farther out than the span of the leaf's other poles, is evaluated
  // directly like the extreme root.
  P->opole = -1;
  P->outlier2 = -1;
  if (nlev > 0) {
    const int la = ((K - 1) / s) * s, fe = std::min(K, s);   // first pole of the last leaf, end of the first
    if (K - la >= 3 && g[K - 1] - g[K - 2] > g[K - 2] - g[la]) {
      P->opole = K - 1;
      const double lim = g[K - 2] + (g[K - 2] - g[la]);
      for (int i = la; i < K; ++i)
        if (i != P->outlier && mu[i] > lim) P->outlier2 = i;
    } else if (fe >= 3 && g[1] - g[0] > g[fe - 1] - g[1]) {
      P->opole = 0;
      const double lim = g[1] - (g[fe - 1] - g[1]);
      for (int i = 0; i < fe; ++i)
        if (i != P->outlier && mu[i] < lim) P->outlier2 = i;
    }
  }
  auto in_box = [&](int i) { return i != P->outlier && i != P->outlier2; };
  P->nlev = nlev;
  P->nbox = (1 << (nlev + 1)) - 1;
  P->lo.assign(P->nbox, 0.0);
  P->hi.assign(P->nbox, 0.0);
  P->s0.assign(P->nbox, 0);
  P->s1.assign(P->nbox, 0);
  P->lev_off.resize(nlev + 2);
  for (int l = 0; l <= nlev + 1; ++l) P->lev_off[l] = (1 << l) - 1;
  for (int b = 0; b < (1 << nlev); ++b) {
    const int id = fmm_box_id(nlev, b);
    const int a0 = std::min(K, b * s), a1 = std::min(K, (b + 1) * s);
    P->s0[id] = a0;
    P->s1[id] = a1;
    if (a0 < a1) {
      const int f = (a0 == P->opole && a1 > a0 + 1) ? a0 + 1 : a0;
      double lo = g[f], hi = g[f];
      for (int i = a0; i < a1; ++i) {
        if (i != P->opole) {
          lo = std::min(lo, g[i]);
          hi = std::max(hi, g[i]);
        }
        if (in_box(i)) {
          lo = std::min(lo, mu[i]);
          hi = std::max(hi, mu[i]);
        }
      }
      P->lo[id] = lo;
      P->hi[id] = hi;
    }
  }
  for (int l = nlev - 1; l >= 0; --l) {
    for (int b = 0; b < (1 << l); ++b) {
      const int id = fmm_box_id(l, b), c0 = fmm_box_id(l + 1, 2 * b), c1 = fmm_box_id(l + 1, 2 * b + 1);
      P->s0[id] = P->s0[c0];
      P->s1[id] = std::max(P->s1[c0], P->s1[c1]);
      if (P->s1[c1] > P->s0[c1] && P->s1[c0] > P->s0[c0]) {
        P->lo[id] = std::min(P->lo[c0], P->lo[c1]);
        P->hi[id] = std::max(P->hi[c0], P->hi[c1]);
      } else if (P->s1[c0] > P->s0[c0]) {
        P->lo[id] = P->lo[c0];
        P->hi[id] = P->hi[c0];
      }
      if (P->s1[c1] > P->s0[c1] && P->s1[c0] <= P->s0[c0]) P->s0[id] = P->s0[c1];
    }
  }
  // dual traversal: M2L lists for every box, near lists for leaves
  std::vector<std::vector<int>> m2l(P->nbox), nearl(P->nbox);
  auto empty = [&](int id) { return P->s1[id] <= P->s0[id]; };
  auto adm = [&](int a, int b) {
    if (a == b) return false;
    const double wa = P->hi[a] - P->lo[a], wb = P->hi[b] - P->lo[b];
    const double gap = std::max(P->lo[b] - P->hi[a], P->lo[a] - P->hi[b]);
    return gap > 0.0 && gap >= std::max(wa, wb);
  };
  std::vector<std::pair<int, int>> stack;
  stack.push_back({0, 0});
  std::vector<int> level_of(P->nbox);
  for (int l = 0; l <= nlev; ++l)
    for (int b = 0; b < (1 << l); ++b) level_of[fmm_box_id(l, b)] = l;
  while (!stack.empty()) {
    auto [a, b] = stack.back();
    stack.pop_back();
    if (empty(a) || empty(b)) continue;
    if (adm(a, b)) {
      m2l[a].push_back(b);
      continue;
    }
    const int l = level_of[a];
    if (l == nlev) {
      nearl[a].push_back(b);
      continue;
    }
    const int ka = a - P->lev_off[l], kb = b - P->lev_off[l];
    for (int ca = 0; ca < 2; ++ca)
      for (int cb = 0; cb < 2; ++cb) stack.push_back({fmm_box_id(l + 1, 2 * ka + ca), fmm_box_id(l + 1, 2 * kb + cb)});
  }
  P->m2l_ptr.assign(P->nbox + 1, 0);
  P->near_ptr.assign(P->nbox + 1, 0);
  for (int i = 0; i < P->nbox; ++i) {
    std::sort(m2l[i].begin(), m2l[i].end());
    std::sort(nearl[i].begin(), nearl[i].end());
    P->m2l_ptr[i + 1] = P->m2l_ptr[i] + (int)m2l[i].size();
    P->near_ptr[i + 1] = P->near_ptr[i] + (int)nearl[i].size();
  }
  P->m2l_src.clear();
  P->near_src.clear();
  for (int i = 0; i < P->nbox; ++i) {
    P->m2l_src.insert(P->m2l_src.end(), m2l[i].begin(), m2l[i].end());
    P->near_src.insert(P->near_src.end(), nearl[i].begin(), nearl[i].end());
  }
  // Each directly evaluated root y takes the far field of every box whose gap
  // to y is at least the box's width (the rule of the pairs above, for a
  // point) from its multipole coefficients, and sums the leaves that never
  // qualify exactly.
  P->dm2p.clear();
  P->dp2p.clear();
  int nd = 0;
  for (const int d : {P->outlier, P->outlier2}) {
    if (d < 0) continue;
    const double y = mu[d];
    std::vector<int> st{0};
    while (!st.empty()) {
      const int b = st.back();
      st.pop_back();
      if (empty(b)) continue;
      const double gap = std::max(P->lo[b] - y, y - P->hi[b]);
      if (gap > 0.0 && gap >= P->hi[b] - P->lo[b]) {
        P->dm2p.push_back(b);
        continue;
      }
      const int l = level_of[b];
      if (l == nlev) {
        P->dp2p.push_back(b);
        continue;
      }
      const int kb = b - P->lev_off[l];
      st.push_back(fmm_box_id(l + 1, 2 * kb + 1));
      st.push_back(fmm_box_id(l + 1, 2 * kb));
    }
    ++nd;
    P->dm2p_ptr[nd] = (int)P->dm2p.size();
    P->dp2p_ptr[nd] = (int)P->dp2p.size();
  }
}

}  // namespace svdu
