// One symmetric rank-one eigen-update up to (not including) the product:
// deflation, the secular roots, the eigenvector weights and the descriptors
// of C~. Section 6.2 of the paper (RankOneUpdate Steps 2, 3, 5 and 7),
// Section 3.1 (deflation cases) and equation GolubEigenvalUpdate.
//
// Readings where the paper is silent:
//  * a component z_j is dropped when |z_j| <= 8 u sqrt(N) |z| (rounding noise
//    of a projection); exactly repeated poles merge into one pole whose weight
//    is the norm of their z entries, and a Householder reflection supplies
//    the group's other eigenvectors. Close but distinct poles stay separate.
//  * each root is stored as (origin pole, offset tau), the origin being the
//    nearer pole, so that every difference d_j - mu_i is formed as
//    (d_j - d_origin) - tau without cancellation.
//  * the eigenvector weights are recomputed from the roots (Loewner formula),
//    which keeps C~ orthogonal to working precision.
#include <math.h>

#include <type_traits>

#include "device_util.h"
#include "jobs.h"
#include "svdu_internal.h"

namespace svdu {

// ---------------------------------------------------------------------------
// Deflation: one block of 1024 threads walks the N sorted poles.
// ---------------------------------------------------------------------------
constexpr int kDeflThreads = 1024;
constexpr int kWideCluster = 64;   // larger clusters of equal poles are handled by a whole block
constexpr int kWideMax = 64;       // such clusters listed per block (more: one thread each, as the rest)

__device__ void deflate_body(const Stage& s) {
  __shared__ int shi[64];
  __shared__ double shd[64];
  if (*s.status & kStFatal) return;
  const int N = s.N;
  const int tid = threadIdx.x, nt = blockDim.x;
  double loc = 0.0;
  int bad = 0;
  for (int t = tid; t < N; t += nt) {
    const int j = s.col_of[t];
    const double zz = s.z[j];
    const double dd = s.lam_in[j];
    s.dsort[t] = dd;
    s.zs[t] = zz;
    loc += zz * zz;
    if (!isfinite(dd) || !isfinite(zz)) bad |= kStNonFinite;
    if (t > 0 && !(s.lam_in[s.col_of[t - 1]] <= dd)) bad |= kStBadSigma;
  }
  const double znorm = sqrt(block_sum(loc, shd));
  const double rho = *s.rho;
  if (!isfinite(znorm) || !isfinite(rho) || rho == 0.0) bad |= kStNonFinite;
  // every thread learns whether any thread saw bad data
  __shared__ int shbad;
  if (tid == 0) shbad = 0;
  __syncthreads();
  if (bad) atomicOr(&shbad, bad);
  __syncthreads();
  bad = shbad;
  if (bad) {
    // record the error and describe C~ = I (everything deflated, in order), so
    // that nothing downstream can derive an index from the bad data
    if (tid == 0) {
      atomicOr(s.status, bad);
      s.counts[0] = 0;
      s.counts[1] = N;
      s.counts[2] = 0;
    }
    for (int t = tid; t < N; t += nt) {
      const int j = s.col_of[t];
      s.clu[t] = -1;
      s.dlist[t] = t;
      s.dval[t] = 0.0;
      s.rg[j] = 0.0;
      s.rh[j] = 0.0;
      s.rcl[j] = t;
      s.flags[j] = 1;
    }
    return;
  }
  const double tol = 8.0 * kU * sqrt((double)(N > 0 ? N : 1)) * znorm;
  __syncthreads();
  // kept components -> Llist
  int carry = 0;
  for (int base = 0; base < N; base += nt) {
    const int t = base + tid;
    const bool keep = (t < N) && !(fabs(s.zs[t]) <= tol);
    int tot;
    const int incl = block_scan_incl(keep ? 1 : 0, shi, &tot);
    if (keep) s.Llist[carry + incl - 1] = t;
    if (t < N && !keep) s.clu[t] = -1;
    carry += tot;
  }
  const int Nl = carry;
  __syncthreads();
  // clusters of exactly equal poles among the kept components
  carry = 0;
  for (int base = 0; base < Nl; base += nt) {
    const int k = base + tid;
    bool nc = false;
    if (k < Nl) nc = (k == 0) || (s.dsort[s.Llist[k]] != s.dsort[s.Llist[k - 1]]);
    int tot;
    const int incl = block_scan_incl(nc ? 1 : 0, shi, &tot);
    if (k < Nl) {
      const int cid = carry + incl - 1;
      s.clu[s.Llist[k]] = cid;
      if (nc) s.cfirst[cid] = k;
    }
    carry += tot;
  }
  const int K = carry;
  __shared__ int nwide, wide[kWideMax];
  if (tid == 0) nwide = 0;
  __syncthreads();
  // per cluster: pole, weight, Householder vector, row descriptors of members;
  // a cluster of more than kWideCluster members (the exact zero block of D_v
  // is one) is listed for the whole block instead of one thread
  for (int c = tid; c < K; c += nt) {
    const int f = s.cfirst[c];
    const int e = (c + 1 < K) ? s.cfirst[c + 1] : Nl;
    const int sz = e - f;
    s.csize[c] = sz;
    if (sz > kWideCluster) {
      const int q = atomicAdd(&nwide, 1);
      if (q < kWideMax) {
        wide[q] = c;
        continue;
      }
    }
    const double gc = s.dsort[s.Llist[f]];
    s.g[c] = gc;
    double w2 = 0.0;
    for (int k = f; k < e; ++k) {
      const double zz = s.zs[s.Llist[k]];
      w2 += zz * zz;
    }
    const double w = sqrt(w2);
    s.W2[c] = w2;
    s.W[c] = w;
    double sg = 1.0, hn = 1.0;
    if (sz >= 2) {
      const double v0 = s.zs[s.Llist[f]] / w;
      sg = (v0 >= 0.0) ? 1.0 : -1.0;
      hn = sqrt(2.0 * (1.0 + fabs(v0)));
    }
    for (int k = f; k < e; ++k) {
      const int t = s.Llist[k];
      const int j = s.col_of[t];
      s.rg[j] = gc;
      s.rcl[j] = c;
      s.flags[j] = (k == f) ? 0 : 2;
      s.rh[j] = (sz >= 2) ? (s.zs[t] / w + (k == f ? sg : 0.0)) / hn : 0.0;
    }
  }
  __syncthreads();
  // the listed clusters, each by the whole block (weight by a fixed-order block sum)
  const int nw = min(nwide, kWideMax);
  for (int q = 0; q < nw; ++q) {
    const int c = wide[q];
    const int f = s.cfirst[c];
    const int e = (c + 1 < K) ? s.cfirst[c + 1] : Nl;
    double loc = 0.0;
    for (int k = f + tid; k < e; k += nt) {
      const double zz = s.zs[s.Llist[k]];
      loc += zz * zz;
    }
    const double w2 = block_sum(loc, shd);
    const double w = sqrt(w2);
    const double gc = s.dsort[s.Llist[f]];
    if (tid == 0) {
      s.g[c] = gc;
      s.W2[c] = w2;
      s.W[c] = w;
    }
    const double v0 = s.zs[s.Llist[f]] / w;
    const double sg = (v0 >= 0.0) ? 1.0 : -1.0;
    const double hn = sqrt(2.0 * (1.0 + fabs(v0)));
    for (int k = f + tid; k < e; k += nt) {
      const int t = s.Llist[k];
      const int j = s.col_of[t];
      s.rg[j] = gc;
      s.rcl[j] = c;
      s.flags[j] = (k == f) ? 0 : 2;
      s.rh[j] = (s.zs[t] / w + (k == f ? sg : 0.0)) / hn;
    }
  }
  __syncthreads();
  // deflated list: dropped components and non-first cluster members
  carry = 0;
  for (int base = 0; base < N; base += nt) {
    const int t = base + tid;
    bool dfl = false;
    if (t < N) {
      const int c = s.clu[t];
      dfl = (c < 0) || (s.Llist[s.cfirst[c]] != t);
    }
    int tot;
    const int incl = block_scan_incl(dfl ? 1 : 0, shi, &tot);
    if (dfl) {
      const int kd = carry + incl - 1;
      s.dlist[kd] = t;
      s.dval[kd] = s.dsort[t];
      if (s.clu[t] < 0) {
        const int j = s.col_of[t];
        s.rg[j] = 0.0;
        s.rh[j] = 0.0;
        s.rcl[j] = K + kd;   // a group of its own
        s.flags[j] = 1;
      }
    }
    carry += tot;
  }
  if (tid == 0) {
    s.counts[0] = K;
    s.counts[1] = carry;
    s.counts[2] = Nl;
  }
}

// ---------------------------------------------------------------------------
// Secular equation, one root per wave of 64 lanes (lanes stride over poles).
// Works in the reflected problem when rho < 0 so that the iteration always
// sees rho > 0 and roots to the right of their left pole.
// ---------------------------------------------------------------------------
// The poles and weights are read from global memory, or (LDS) from a copy the
// block staged in LDS; the arithmetic is the same either way.
template <bool LDS>
struct Reflect {
  const double* g;
  const double* W2;
  int K;
  bool refl;
  static __device__ __forceinline__ double ld(const double* p) {
    if (LDS) return *((const __attribute__((address_space(3))) double*)p);
    return gld(p);
  }
  // branch-free (index and sign by select), so loops over k keep several loads in flight
  __device__ __forceinline__ double pole(int k) const {
    const double v = ld(g + (refl ? K - 1 - k : k));
    return refl ? -v : v;
  }
  __device__ __forceinline__ double wt(int k) const { return ld(W2 + (refl ? K - 1 - k : k)); }
};

struct SecSums {
  double psi, dpsi, phi, dphi;
};

// Pole k and its weight z_k^2 of the (reflected) problem, in units of 1 / sc
// when SC (an exact power-of-two scaling).
template <bool REFL, bool SC, bool LDS>
__device__ __forceinline__ void sec_pole(const Reflect<LDS>& R, int k, double sc, double* p, double* wt) {
  const int kk = REFL ? R.K - 1 - k : k;
  const double v = R.ld(R.g + kk), w = R.ld(R.W2 + kk);
  *p = SC ? (REFL ? -v : v) * sc : (REFL ? -v : v);
  *wt = SC ? w * sc : w;
}

// Adds one term w = wt / del to a and w / del to da: times recip_fast(del)
// with an fma for the derivative, or, in the EXACT pass, by true divisions
// where |del| is below recip_fast's range (where 1 / del alone may overflow).
// The fast pass flags such terms in t.
template <bool EXACT>
__device__ __forceinline__ void sec_add(double wt, double del, double* a, double* da, bool* t) {
  if (EXACT && recip_tiny(del)) {
    const double w = wt / del;
    *a += w;
    *da += w / del;
  } else {
    if (!EXACT) *t |= recip_tiny(del);
    const double r = recip_fast(del);
    const double w = wt * r;
    *a += w;
    *da = __builtin_fma(w, r, *da);
  }
}

// Terms k = k0, k0 + STEP, ... < k1 added in increasing k.
template <bool REFL, bool SC, bool EXACT, int STEP, bool LDS>
__device__ inline void secular_range(const Reflect<LDS>& R, double sc, int k0, int k1, double po, double tau,
                                     double* s, double* ds, bool* tiny) {
  double a = *s, da = *ds;
  bool t = false;
#pragma unroll 4
  for (int k = k0; k < k1; k += STEP) {
    double p, wt;
    sec_pole<REFL, SC, LDS>(R, k, sc, &p, &wt);
    sec_add<EXACT>(wt, (p - po) - tau, &a, &da, &t);
  }
  *s = a;
  *ds = da;
  *tiny = *tiny || t;
}

// Sums over poles at x = P(o) + tau: psi/dpsi over poles k <= i, phi/dphi over
// k > i, for a root owned by a group of G lanes. Lane `sub` of the group takes
// k = sub, sub + G, ... in increasing order; the poles k <= i and k > i run as
// two loops and the reflection is a template parameter, so the loops are
// branch-free and keep several loads in flight. A group that meets a |delta|
// below recip_fast's range repeats its sums in the exact form, with the same
// terms in the same order.
template <bool REFL, bool SC, int G, bool LDS>
__device__ inline SecSums secular_sums_t(const Reflect<LDS>& R, double sc, int i, double po, double tau, int sub) {
  double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
  bool tiny = false;
  const int kr = (i + 1) + ((sub - (i + 1)) & (G - 1));   // first k > i with k = sub (mod G)
  secular_range<REFL, SC, false, G, LDS>(R, sc, sub, i + 1, po, tau, &psi, &dpsi, &tiny);
  secular_range<REFL, SC, false, G, LDS>(R, sc, kr, R.K, po, tau, &phi, &dphi, &tiny);
  if (group_any<G>(tiny)) {
    psi = dpsi = phi = dphi = 0.0;
    secular_range<REFL, SC, true, G, LDS>(R, sc, sub, i + 1, po, tau, &psi, &dpsi, &tiny);
    secular_range<REFL, SC, true, G, LDS>(R, sc, kr, R.K, po, tau, &phi, &dphi, &tiny);
  }
  return SecSums{group_sum<G>(psi), group_sum<G>(dpsi), group_sum<G>(phi), group_sum<G>(dphi)};
}

// ---------------------------------------------------------------------------
// Secular sums with the far field from Chebyshev interpolants (the option
// SVDU_OPT_SECULAR_FMM). Section 3.1 of the paper rules the FMM out for the
// secular equation because the evaluation points (the iterates) are not known
// in advance; they are, however, known to stay in the gap of their root, and
// the sources (poles and weights) are fixed. So the far field is sampled
// once per eigen-update around the gaps, in the spirit of the fast multipole
// method, and every iterate evaluates it in O(p):
//  * the poles of the (reflected) problem fall into leaves of kSfLeaf
//    consecutive poles. Leaf l's interval T runs from its first pole to the
//    first pole of the next leaf (the last leaf: to the last pole), so every
//    root of the leaf lies in T. Two roots are solved with the direct sums
//    instead: the extreme root beyond the last pole (its interval, up to
//    d_{K-1} + rho sum w, can be wider than all the poles together) and the
//    root between the first two poles (after an update with rho > 0 the top
//    eigenvalue can sit far above the rest, and the next update, with
//    rho < 0, sees it reflected as its first pole). Leaf 0 starts at pole 1;
//  * a pole at distance >= |T| from T is far. Far poles left of T are all
//    below every root of the leaf (they enter psi), far poles right of it all
//    above (they enter phi). Each of psi, psi', phi, phi' over the far poles
//    is analytic around T with its nearest singularity |T| away, so its
//    interpolant at kSfP Chebyshev points of T converges like (3 + sqrt 8)^-p;
//    it is evaluated in the barycentric form from the node values, which
//    keeps its rounding at a few units (the coefficient form loses about p);
//  * the near poles form one contiguous range [kl, kr] (the leaf and its
//    neighbours within |T|), summed directly with the pole-relative
//    differences of the direct form.
// Nodes and evaluation points are formed as offsets from the leaf's first
// pole, so a leaf far from the origin keeps its relative resolution.
// ---------------------------------------------------------------------------
constexpr int kSfP = 32;      // Chebyshev points of the far-field interpolants (kSfLeaf poles per leaf)

struct SfLeaf {
  double h, hinv;       // half-width of T and its reciprocal
  int k0, kl, kr;       // first pole of the leaf; near range [kl, kr]
  double t[kSfP];       // Chebyshev points of the first kind on [-1, 1]
  double lam[kSfP];     // their barycentric weights (-1)^q sin((2q + 1) pi / 2p)
  double f[4][kSfP];    // psi, psi', phi, phi' of the far poles at the points
};

// Sums at x = po + tau as secular_sums_t, with the poles outside [kl, kr]
// taken from the leaf's interpolants: lane `sub` of the group adds points sub
// and sub + 16 to the barycentric numerators and denominator.
template <bool REFL, bool SC, int G, bool LDS>
__device__ inline SecSums secular_sums_ff(const Reflect<LDS>& R, double sc, int i, double po, double tau, int sub,
                                          const SfLeaf& f, double plo) {
  static_assert(G == 16 && kSfP == 2 * G, "two interpolation points per lane");
  double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
  bool tiny = false;
  secular_range<REFL, SC, false, G, LDS>(R, sc, f.kl + sub, i + 1, po, tau, &psi, &dpsi, &tiny);
  secular_range<REFL, SC, false, G, LDS>(R, sc, i + 1 + sub, f.kr + 1, po, tau, &phi, &dphi, &tiny);
  if (group_any<G>(tiny)) {
    psi = dpsi = phi = dphi = 0.0;
    secular_range<REFL, SC, true, G, LDS>(R, sc, f.kl + sub, i + 1, po, tau, &psi, &dpsi, &tiny);
    secular_range<REFL, SC, true, G, LDS>(R, sc, i + 1 + sub, f.kr + 1, po, tau, &phi, &dphi, &tiny);
  }
  // the iterate in the coordinate of T, from offsets to the leaf's first pole
  const double t = (((po - plo) + tau) - f.h) * f.hinv;
  double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0, den = 0.0;
  const double dt0 = t - f.t[sub], dt1 = t - f.t[sub + G];
  // Within 2^-60 of a point (in the coordinate of T, where every far sum
  // changes by at most half its size per unit) that point's values are the
  // result to far below rounding, and the quotient below could overflow.
  const bool hit0 = fabs(dt0) < 0x1p-60, hit1 = fabs(dt1) < 0x1p-60;
  if (group_any<G>(hit0 || hit1)) {
    const int q = hit0 ? sub : sub + G;
    const bool h = hit0 || hit1;
    n0 = h ? f.f[0][q] : 0.0;
    n1 = h ? f.f[1][q] : 0.0;
    n2 = h ? f.f[2][q] : 0.0;
    n3 = h ? f.f[3][q] : 0.0;
    den = h ? 1.0 : 0.0;
  } else {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int q = sub + e * G;
      const double r = f.lam[q] * recip_fast(e == 0 ? dt0 : dt1);
      n0 = __builtin_fma(r, f.f[0][q], n0);
      n1 = __builtin_fma(r, f.f[1][q], n1);
      n2 = __builtin_fma(r, f.f[2][q], n2);
      n3 = __builtin_fma(r, f.f[3][q], n3);
      den += r;
    }
  }
  den = group_sum<G>(den);
  const double dinv = 1.0 / den;
  return SecSums{group_sum<G>(psi) + group_sum<G>(n0) * dinv, group_sum<G>(dpsi) + group_sum<G>(n1) * dinv,
                 group_sum<G>(phi) + group_sum<G>(n2) * dinv, group_sum<G>(dphi) + group_sum<G>(n3) * dinv};
}

// A power of two near |x| (x finite and nonzero), else 1. Lengths divided by it
// and derivatives multiplied by it scale exactly, so the quadratics below keep
// their coefficients at the scale of the secular function itself: without it
// products of two pole distances underflow once the poles are below about
// 2^-511 (and overflow above 2^511).
__device__ inline double length_unit(double x) {
  if (!(x != 0.0) || !isfinite(x)) return 1.0;
  return ldexp(1.0, ilogb(x));
}

// The unit S of the secular iteration: a power of two near the largest |pole|
// when that lies outside [2^-500, 2^500], else 1. Poles and weights divided by
// S (exactly) keep every sum and quadratic away from overflow and underflow;
// the roots are scaled back at the end.
template <bool LDS>
__device__ inline double secular_unit(const Reflect<LDS>& R) {
  const double pmax = fmax(fabs(R.ld(R.g)), fabs(R.ld(R.g + R.K - 1)));   // the poles ascend
  const bool scaled = pmax != 0.0 && (pmax < 0x1p-500 || pmax > 0x1p500);
  return scaled ? fmax(length_unit(pmax), 0x1p-1000) : 1.0;
}

// Root of c x^2 - a x + b = 0 inside (lo, hi); returns false when none is.
__device__ inline bool quad_root_in(double c, double a, double b, double lo, double hi, double* x) {
  double r1, r2;
  if (c == 0.0) {
    if (a == 0.0) return false;
    r1 = r2 = b / a;
  } else {
    double disc = a * a - 4.0 * b * c;
    if (disc < 0.0) disc = 0.0;
    const double q = 0.5 * (a + copysign(sqrt(disc), a));
    if (q == 0.0) return false;
    r1 = q / c;
    r2 = b / q;
  }
  const bool in1 = (r1 > lo) && (r1 < hi);
  const bool in2 = (r2 > lo) && (r2 < hi);
  if (in1 && in2) {
    *x = (fabs(r1) < fabs(r2)) ? r1 : r2;
    return true;
  }
  if (in1) { *x = r1; return true; }
  if (in2) { *x = r2; return true; }
  return false;
}

// One root: the midpoint two-pole start, then middle-way steps safeguarded
// by bisection. Root `idx` belongs to an aligned group of G lanes of the wave
// (G = 64: the whole wave), which splits the sums over its lanes; every lane
// of the group takes the same decisions from the same reduced sums.
// FF: the sums take their far field from the leaf `lf` (secular_sums_ff).
template <int G, bool LDS, bool FF = false>
__device__ void secular_body(const int* __restrict__ Kdev, const double* __restrict__ g,
                             const double* __restrict__ W2, const double* __restrict__ rhop,
                             int* __restrict__ org, double* __restrict__ tau_out, int* __restrict__ iters,
                             int* status, int maxit, int idx, const SfLeaf* lf = nullptr) {
  if (*status & kStFatal) return;
  const int K = *Kdev;
  const int sub = threadIdx.x & (G - 1);
  if (idx >= K) return;
  const double rho0 = *rhop;
  Reflect<LDS> R{g, W2, K, rho0 < 0.0};
  const double rho = fabs(rho0);
  const double rinv = 1.0 / rho;
  const int i = R.refl ? K - 1 - idx : idx;  // root index in the reflected problem
  // work in units of S (secular_unit); in between S = 1 and nothing is rescaled
  const double S = secular_unit(R);
  const bool scaled = S != 1.0;
  const double sc = 1.0 / S;
  auto pole = [&](int k) { return R.pole(k) * sc; };
  auto wt = [&](int k) { return R.wt(k) * sc; };
  const double plo = FF ? pole(lf->k0) : 0.0;
  auto sums = [&](double po, double tau) -> SecSums {
    if constexpr (FF) {
      if (scaled)
        return R.refl ? secular_sums_ff<true, true, G, LDS>(R, sc, i, po, tau, sub, *lf, plo)
                      : secular_sums_ff<false, true, G, LDS>(R, sc, i, po, tau, sub, *lf, plo);
      return R.refl ? secular_sums_ff<true, false, G, LDS>(R, sc, i, po, tau, sub, *lf, plo)
                    : secular_sums_ff<false, false, G, LDS>(R, sc, i, po, tau, sub, *lf, plo);
    } else {
      if (scaled)
        return R.refl ? secular_sums_t<true, true, G, LDS>(R, sc, i, po, tau, sub)
                      : secular_sums_t<false, true, G, LDS>(R, sc, i, po, tau, sub);
      return R.refl ? secular_sums_t<true, false, G, LDS>(R, sc, i, po, tau, sub)
                    : secular_sums_t<false, false, G, LDS>(R, sc, i, po, tau, sub);
    }
  };

  int o;
  double lo, hi, tau;
  if (i < K - 1) {
    const double pi = pole(i), pi1 = pole(i + 1);
    const double gap = pi1 - pi;
    const double half = 0.5 * gap;
    const SecSums m = sums(pi, half);
    const double fmid = rinv + m.psi + m.phi;
    const double qi = wt(i), qi1 = wt(i + 1);
    // two-pole model at the midpoint: c + qi/(pi - x) + qi1/(pi1 - x)
    const double c = fmid + qi / half - qi1 / half;
    // the same model in units of sg (exact scaling; see length_unit)
    const double sg = length_unit(gap);
    const double gs = gap / sg, qs = qi / sg, q1s = qi1 / sg;
    double a, b;
    if (fmid >= 0.0) {
      o = i;
      lo = 0.0;
      hi = half;
      a = c * gs + qs + q1s;
      b = qs * gs;
    } else {
      o = i + 1;
      lo = -half;
      hi = 0.0;
      a = -c * gs + qs + q1s;
      b = -q1s * gs;
    }
    double ts = 0.0;
    tau = quad_root_in(c, a, b, lo / sg, hi / sg, &ts) ? ts * sg : 0.5 * (lo + hi);
    if (fmid == 0.0) tau = (o == i) ? half : -half;
  } else {
    o = K - 1;
    double w = 0.0;
    for (int k = sub; k < K; k += G) w += wt(k);
    w = group_sum<G>(w);
    lo = 0.0;
    hi = rho * w;
    tau = 0.5 * hi;
  }
  const double po = pole(o);
  const double dl = pole(i) - po;                          // left pole offset
  const double dr = (i < K - 1) ? (pole(i + 1) - po) : 0.0;  // right pole offset
  bool done = false;
  int it = 0;
  for (; it < maxit; ++it) {
    const SecSums s = sums(po, tau);
    const double f = rinv + s.psi + s.phi;
    if (f < 0.0) lo = tau; else hi = tau;
    const double err = 8.0 * (s.phi - s.psi) + 2.0 * rinv + 3.0 * fabs(f) + fabs(tau) * (s.dpsi + s.dphi);
    if (fabs(f) <= kU * err || f == 0.0) { done = true; break; }
    if (hi - lo <= 4.0 * kU * fmax(fabs(lo), fabs(hi))) { done = true; break; }
    double eta;
    bool ok;
    const double dL = dl - tau;
    if (i < K - 1) {
      // the middle-way quadratic in units of su (exact scaling; see length_unit)
      const double dR = dr - tau;
      const double su = length_unit(fmax(fabs(dL), fabs(dR)));
      const double dLs = dL / su, dRs = dR / su, dps = s.dpsi * su, dfs = s.dphi * su;
      const double c = f - dLs * dps - dRs * dfs;
      const double a = f * (dLs + dRs) - dLs * dRs * (dps + dfs);
      const double b = dLs * dRs * f;
      double es = 0.0;
      ok = quad_root_in(c, a, b, (lo - tau) / su, (hi - tau) / su, &es);
      eta = es * su;
    } else {
      const double su = length_unit(dL);
      const double dLs = dL / su, dps = s.dpsi * su;
      const double c = f - dLs * dps;
      ok = c > 0.0;
      eta = ok ? (dLs + dLs * dLs * dps / c) * su : 0.0;
    }
    if (!ok || f * eta >= 0.0) eta = -f / (s.dpsi + s.dphi);
    double tn = tau + eta;
    if (!(tn > lo && tn < hi) || it >= 40) tn = 0.5 * (lo + hi);
    if (tn == tau) { done = true; break; }
    tau = tn;
  }
  if (!isfinite(tau)) {  // keeps mu inside its interval whatever happened
    tau = 0.0;
    done = false;
  }
  if (sub == 0) {
    if (!done) atomicOr(status, (int)kStNoConv);
    const int ow = R.refl ? K - 1 - o : o;
    org[idx] = ow;
    tau_out[idx] = (R.refl ? -tau : tau) * S;
    if (iters) iters[idx] = it + 1;
  }
}

// ---------------------------------------------------------------------------
// Loewner weights, reflected for rho<0:
// |w_j|^2 = prod_i (mu_i - d_j) / (rho prod_{k != j} (d_k - d_j)), as K ratios
// in (0, 1] pairing root i with pole i (i < j) or i+1 (i >= j), last with rho.
// Pole `idx` belongs to an aligned group of G lanes (lanes over roots).
// ---------------------------------------------------------------------------
template <int G, bool LDS>
__device__ void loewner_body(const int* __restrict__ Kdev, const double* __restrict__ g,
                             const double* __restrict__ rhop, const int* __restrict__ org,
                             const double* __restrict__ tau, double* __restrict__ what, const int* status,
                             int idx) {
  if (*status & kStFatal) return;
  const int K = *Kdev;
  const int lane = threadIdx.x & 63;
  if (idx >= K) return;
  const int k0 = lane & (G - 1), step = G;
  const double rho0 = *rhop;
  const bool refl = rho0 < 0.0;
  const double rho = fabs(rho0);
  Reflect<LDS> R{g, nullptr, K, refl};
  const int jr = refl ? K - 1 - idx : idx;  // pole index in the reflected problem
  const double pj = R.pole(jr);
  double prod = 1.0;
#pragma unroll 4
  for (int ir = k0; ir < K; ir += step) {   // branch-free body
    const int io = refl ? K - 1 - ir : ir;
    const int o = gld(org + io);
    const double tv = gld(tau + io);
    const int orr = refl ? K - 1 - o : o;
    const double tr = refl ? -tv : tv;
    const double num = (R.pole(orr) - pj) + tr;
    const int pr = (ir < jr) ? ir : (ir + 1 < K ? ir + 1 : K - 1);
    const double den = (ir == K - 1) ? rho : (R.pole(pr) - pj);
    prod *= num / den;
  }
  prod = group_prod<G>(prod);
  if (k0 == 0) what[idx] = sqrt(fabs(prod));
}

// ---------------------------------------------------------------------------
// Column scales 1/|c_i| with |c_i|^2 = sum_k what_k^2 / delta_ki^2, and mu.
// Root i belongs to an aligned group of G lanes (lanes over poles).
// ---------------------------------------------------------------------------
template <int G, bool LDS>
__device__ void colnorm_body(const int* __restrict__ Kdev, const double* __restrict__ g,
                             const double* __restrict__ what, const int* __restrict__ org,
                             const double* __restrict__ tau, double* __restrict__ cs, double* __restrict__ mu,
                             const int* status, int i) {
  if (*status & kStFatal) return;
  const int K = *Kdev;
  const int lane = threadIdx.x & 63;
  if (i >= K) return;
  const int k0 = lane & (G - 1), step = G;
  auto ld = [](const double* p) { return Reflect<LDS>::ld(p); };   // poles and weights: LDS copy or global
  const double go = ld(g + org[i]);
  const double ti = tau[i];
  // One branch-free pass for the largest term and the unscaled sum of
  // squares. With the largest term in [2^-450, 2^450] no square overflows and
  // any that underflows is negligible; otherwise, or if a |delta| is below
  // recip_fast's range, the wave takes two exact passes, scaled by the largest
  // term.
  double mx = 0.0, ss = 0.0;
  bool tiny = false;
#pragma unroll 4
  for (int k = k0; k < K; k += step) {
    const double del = (ld(g + k) - go) - ti;
    tiny |= recip_tiny(del);
    const double t = ld(what + k) * recip_fast(del);
    mx = fmax(mx, fabs(t));
    ss = __builtin_fma(t, t, ss);
  }
  mx = group_max<G>(mx);
  const bool scaled = group_any<G>(tiny) || !(mx >= 0x1p-450 && mx <= 0x1p450);
  double inv = 1.0;
  if (scaled) {
    mx = 0.0;
    for (int k = k0; k < K; k += step) mx = fmax(mx, fabs(div_by(ld(what + k), (ld(g + k) - go) - ti)));
    mx = group_max<G>(mx);
    inv = (mx > 0.0) ? 1.0 / mx : 1.0;
    ss = 0.0;
    for (int k = k0; k < K; k += step) {
      const double t = div_by(ld(what + k), (ld(g + k) - go) - ti) * inv;
      ss += t * t;
    }
  }
  ss = group_sum<G>(ss);
  if (k0 == 0) {
    cs[i] = (mx > 0.0) ? inv / sqrt(ss) : 0.0;
    mu[i] = go + ti;
  }
}

// ---------------------------------------------------------------------------
// Output positions and descriptors: merge the ascending roots with the
// ascending deflated eigenvalues (ties: root first), then write the column
// descriptors at their output positions and the per-row weights zeta.
// ---------------------------------------------------------------------------
__device__ inline int count_less(const double* a, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ inline int count_leq(const double* a, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ void merge_body(const Stage& s, int idx) {
  if (*s.status & kStFatal) return;
  const int N = s.N;
  const int K = s.counts[0], Kd = s.counts[1];
  if (idx < N) {
    // row weight zeta_j = what_c z_j / W_c (zero for dropped components)
    const int t = idx;
    const int j = s.col_of[t];
    const int c = s.clu[t];
    s.rzeta[j] = (c >= 0) ? s.what[c] * (s.zs[t] / s.W[c]) : 0.0;
  }
  if (idx < K) {
    const double v = s.mu[idx];
    const int pos = idx + count_less(s.dval, Kd, v);
    const int P = s.descending ? N - 1 - pos : pos;
    s.rootpos[idx] = P;
    s.lam_out[P] = v;
    s.ctype[P] = 0;
    s.co[P] = s.g[s.org[idx]];
    s.ctau[P] = s.tau[idx];
    s.ccs[P] = s.cs[idx];
    s.ccl[P] = -1;
    s.cmem[P] = -1;
    s.ch[P] = 0.0;
  } else if (idx < K + Kd) {
    const int kd = idx - K;
    const double v = s.dval[kd];
    const int pos = kd + count_leq(s.mu, K, v);
    const int P = s.descending ? N - 1 - pos : pos;
    const int t = s.dlist[kd];
    const int j = s.col_of[t];
    s.dpos[kd] = P;
    s.lam_out[P] = v;
    s.ctype[P] = 1;
    s.co[P] = 0.0;
    s.ctau[P] = 0.0;
    s.ccs[P] = 0.0;
    s.ccl[P] = s.rcl[j];
    s.cmem[P] = j;
    s.ch[P] = s.rh[j];
  }
}

// ---------------------------------------------------------------------------
// Level kernels: each serves every eigen-update of a level.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kDeflThreads) void deflate_kernel(StageLevel L) {
  const Stage s = L.st[blockIdx.x];
  if (s.N > 0) deflate_body(s);
}

// Item kernels: problems with N <= kGroupMaxN give each item a group of
// kSmallGroup lanes (256 / kSmallGroup items per 256 threads), larger ones a
// whole wave (4 per 256 threads); the host sizes boff_i (256-thread blocks)
// and boff_s (1024-thread blocks, four of those) to match.

// Poles and weights are copied into LDS before the sums, so that every sum
// reads them there rather than through the vector memory path, which bounded
// the global form. A level whose orders are all at most kGroupMaxN runs in
// 256-thread blocks (boff_i) with room for kGroupMaxN poles; otherwise a block
// is four such item blocks of one job (boff_s, 1024 threads) with room for
// kSecLdsN poles, and larger orders read global memory. The item layout and
// every root's arithmetic are those of the 256-thread item kernels.
constexpr int kSecLdsN = 8192;

template <int G, bool LDS>
__device__ __forceinline__ void secular_item(const Stage& s, const double* g, const double* W2, int maxit, int b,
                                             int t) {
  const int item = G == 64 ? b * 4 + (t >> 6) : b * (256 / kSmallGroup) + t / kSmallGroup;
  secular_body<G, LDS>(s.counts, g, W2, s.rho, s.org, s.tau, s.iters, s.status, maxit, item);
}

template <int BT>
__global__ __launch_bounds__(BT) void secular_kernel(StageLevel L, int maxit) {
  constexpr int CAP = BT == 1024 ? kSecLdsN : kGroupMaxN;
  __shared__ double sm[2 * CAP];   // poles, then weights
  const int* boff = BT == 1024 ? L.boff_s : L.boff_i;
  const int j = find_job(boff, L.n, blockIdx.x);
  const Stage s = L.st[j];
  const int b = (blockIdx.x - boff[j]) * (BT / 256) + (threadIdx.x >> 8), t = threadIdx.x & 255;
  if (s.N <= CAP) {
    const int K = min(max(*s.counts, 0), s.N);
    for (int e = threadIdx.x; e < K; e += blockDim.x) {
      sm[e] = gld(s.g + e);
      sm[CAP + e] = gld(s.W2 + e);
    }
    __syncthreads();
    if (s.N <= kGroupMaxN)
      secular_item<kSmallGroup, true>(s, sm, sm + CAP, maxit, b, t);
    else
      secular_item<64, true>(s, sm, sm + CAP, maxit, b, t);
  } else {
    secular_item<64, false>(s, s.g, s.W2, maxit, b, t);
  }
}

// Far-field form of the secular kernel, for levels with an order above
// kGroupMaxN: one block of kSfThreads per leaf, then one more per job for the
// two roots of the direct sums. A leaf's block first builds the leaf's
// interval, near range and interpolation data (sf_setup), then its
// kSfThreads / 16 = kSfLeaf groups of 16 lanes solve the leaf's roots with
// secular_sums_ff. The last block solves the extreme root (wave 0) and the
// root between the first two poles (wave 1) with the direct sums, from an LDS
// copy of the poles as in the secular kernel.
constexpr int kSfThreads = 1024;
static_assert(kSfThreads / 16 == kSfLeaf && kSmallGroup == 16, "one 16-lane group per root of a leaf");
static_assert(kSfThreads == 32 * kSfP, "one thread per (point, pole stride) pair");

// Interval T = [pole a, pole b] (a < b), near range and interpolation data of
// a leaf of the stage's reflected problem (K live poles), in units of the
// secular iteration. The poles pass through LDS in chunks of kSfChunk; each is
// classified on the way (far below T, far above T, or near) and its far terms
// are added at the 32 points. The poles ascend, so the far poles below T are
// the first nl and those above it the last nr, and the near range is
// [nl, K - 1 - nr]. LDS: red 4 * 32 * 33 doubles, sp and sw kSfChunk doubles
// each, cnt 2 ints.
constexpr int kSfChunk = 2048;
constexpr int kSfRed = 4 * 32 * 33;

__device__ void sf_setup(const Stage& s, int K, int a, int b, SfLeaf* lf, double* red, double* sp, double* sw,
                         int* cnt) {
  const double rho0 = *s.rho;
  const Reflect<false> R{s.g, s.W2, K, rho0 < 0.0};
  const double sc = 1.0 / secular_unit(R);
  auto pole = [&](int k) { return R.pole(k) * sc; };
  auto wt = [&](int k) { return R.wt(k) * sc; };
  const int t = threadIdx.x;
  const double lo = pole(a);
  if (t < 2) cnt[t] = 0;
  const double w = pole(b) - lo;
  // far sums at the Chebyshev points x_q = lo + h (1 + t_q): point q = t % 32,
  // poles j = t / 32, t / 32 + 32, ... of each chunk
  const int q = t & (kSfP - 1), r = t >> 5;
  const double tq = cospi((double)(2 * q + 1) / (2.0 * kSfP));
  const double xo = 0.5 * w * (1.0 + tq);
  double s0, s1, s2, s3;
  int nl, nr;
  // One pass over the poles. The fast pass takes every reciprocal from
  // recip_fast, with no branch per pole; if any |D| of the block is below its
  // range (a far pole is at least |T| away, so only for |T| near 2^-1000) the
  // block repeats the pass with true divisions for those.
  auto pass = [&](auto EXACT) {
    s0 = s1 = s2 = s3 = 0.0;
    nl = nr = 0;
    bool tiny = false;
    for (int c0 = 0; c0 < K; c0 += kSfChunk) {
      const int n = min(kSfChunk, K - c0);
      __syncthreads();   // the previous chunk is consumed
      for (int j = t; j < n; j += kSfThreads) {
        sp[j] = pole(c0 + j);
        sw[j] = wt(c0 + j);
      }
      __syncthreads();
#pragma unroll 4
      for (int j = r; j < n; j += 32) {
        const double off = sp[j] - lo;
        const bool fl = off <= -w, fr = off >= 2.0 * w;
        const bool far = fl || fr;
        const double D = far ? off - xo : 1.0;   // far: |D| >= |T|
        double rd;
        if constexpr (decltype(EXACT)::value) {
          rd = far ? (recip_tiny(D) ? 1.0 / D : recip_fast(D)) : 0.0;
        } else {
          tiny |= recip_tiny(D);
          rd = far ? recip_fast(D) : 0.0;
        }
        const double v = sw[j] * rd;
        const double dv = v * rd;
        s0 += fl ? v : 0.0;
        s1 += fl ? dv : 0.0;
        s2 += fr ? v : 0.0;
        s3 += fr ? dv : 0.0;
        nl += fl ? 1 : 0;
        nr += fr ? 1 : 0;
      }
    }
    return tiny;
  };
  if (__syncthreads_or(pass(std::false_type{}))) pass(std::true_type{});
  red[(0 * 32 + r) * 33 + q] = s0;
  red[(1 * 32 + r) * 33 + q] = s1;
  red[(2 * 32 + r) * 33 + q] = s2;
  red[(3 * 32 + r) * 33 + q] = s3;
  if (q == 0) {   // every pole was seen by the 32 threads of one r; count it once
    atomicAdd(&cnt[0], nl);
    atomicAdd(&cnt[1], nr);
  }
  if (r == 0) {
    lf->t[q] = tq;
    const double sq = sinpi((double)(2 * q + 1) / (2.0 * kSfP));
    lf->lam[q] = (q & 1) ? -sq : sq;
  }
  __syncthreads();
  if (t < 4 * kSfP) {
    const int a = t >> 5, qq = t & 31;
    double f = 0.0;
    for (int v = 0; v < 32; ++v) f += red[(a * 32 + v) * 33 + qq];
    lf->f[a][qq] = f;
  }
  if (t == 0) {
    lf->k0 = a;
    lf->kl = cnt[0];
    lf->kr = K - 1 - cnt[1];
    lf->h = 0.5 * w;
    lf->hinv = 2.0 / w;
  }
  __syncthreads();
}

static_assert(kSfRed + 2 * kSfChunk <= 2 * kSecLdsN, "the setup's LDS fits the pole copy's");

// direct_max: jobs of order up to this take the direct sums.
__global__ __launch_bounds__(kSfThreads) void secular_ff_kernel(StageLevel L, int maxit, int direct_max) {
  __shared__ double lds[2 * kSecLdsN];   // setup: red, sp, sw; extreme root: poles, then weights
  __shared__ int cnt[2];
  __shared__ SfLeaf lf;
  const int j = find_job(L.boff_l, L.n, blockIdx.x);
  const Stage s = L.st[j];
  if (*s.status & kStFatal) return;   // set before this launch only: uniform over the block
  const int K = min(max(*s.counts, 0), s.N);
  if (K <= 0) return;
  const int b = blockIdx.x - L.boff_l[j];
  if (s.N <= direct_max) {
    // orders up to kGroupMaxN (direct_max) keep the direct sums with the item
    // layout of secular_kernel (groups of kSmallGroup lanes, 64 roots per
    // block), so a problem's roots do not depend on what shares the launch
    if (b * kSfLeaf >= K) return;
    for (int e = threadIdx.x; e < K; e += blockDim.x) {
      lds[e] = gld(s.g + e);
      lds[kSecLdsN + e] = gld(s.W2 + e);
    }
    __syncthreads();
    secular_body<kSmallGroup, true>(s.counts, lds, lds + kSecLdsN, s.rho, s.org, s.tau, s.iters, s.status, maxit,
                                    b * kSfLeaf + (int)(threadIdx.x / kSmallGroup));
    return;
  }
  const bool refl = *s.rho < 0.0;
  if (b == (s.N + kSfLeaf - 1) / kSfLeaf) {
    // the direct sums: wave 0 the extreme root K - 1, wave 1 root 0 (roots of the reflected problem)
    const int w = threadIdx.x >> 6;
    const int i = w == 0 ? K - 1 : 0;
    const bool mine = w < 2 && (w == 0 || K > 1);
    const int idx = refl ? K - 1 - i : i;
    if (s.N <= kSecLdsN) {
      for (int e = threadIdx.x; e < K; e += blockDim.x) {
        lds[e] = gld(s.g + e);
        lds[kSecLdsN + e] = gld(s.W2 + e);
      }
      __syncthreads();
      if (mine)
        secular_body<64, true>(s.counts, lds, lds + kSecLdsN, s.rho, s.org, s.tau, s.iters, s.status, maxit, idx);
    } else if (mine) {
      secular_body<64, false>(s.counts, s.g, s.W2, s.rho, s.org, s.tau, s.iters, s.status, maxit, idx);
    }
    return;
  }
  // this leaf's roots of the far-field form: [r0, r1) without 0 and K - 1
  const int k0 = b * kSfLeaf;
  const int r0 = max(k0, 1), r1 = min(k0 + kSfLeaf, K - 1);
  if (r0 >= r1) return;
  sf_setup(s, K, r0, r1, &lf, lds, lds + kSfRed, lds + kSfRed + kSfChunk, cnt);
  const int i = k0 + (threadIdx.x >> 4);   // root of the reflected problem
  if (s.N <= kSecLdsN) {
    // the setup's LDS is free again (sf_setup ends with a barrier): the
    // iterates read every pole and weight from an LDS copy, as the direct sums do
    for (int e = threadIdx.x; e < K; e += blockDim.x) {
      lds[e] = gld(s.g + e);
      lds[kSecLdsN + e] = gld(s.W2 + e);
    }
    __syncthreads();
    if (i < r0 || i >= r1) return;
    secular_body<16, true, true>(s.counts, lds, lds + kSecLdsN, s.rho, s.org, s.tau, s.iters, s.status, maxit,
                                 refl ? K - 1 - i : i, &lf);
    return;
  }
  if (i < r0 || i >= r1) return;
  secular_body<16, false, true>(s.counts, s.g, s.W2, s.rho, s.org, s.tau, s.iters, s.status, maxit,
                                refl ? K - 1 - i : i, &lf);
}

// Block shapes and the LDS copy of the poles as in the secular kernel; the
// roots' origins and offsets stream from global memory.
template <int BT>
__global__ __launch_bounds__(BT) void loewner_kernel(StageLevel L) {
  constexpr int CAP = BT == 1024 ? kSecLdsN : kGroupMaxN;
  __shared__ double sg[CAP];
  const int* boff = BT == 1024 ? L.boff_s : L.boff_i;
  const int j = find_job(boff, L.n, blockIdx.x);
  const Stage s = L.st[j];
  const int b = (blockIdx.x - boff[j]) * (BT / 256) + (threadIdx.x >> 8), t = threadIdx.x & 255;
  if (s.N <= CAP) {
    const int K = min(max(*s.counts, 0), s.N);
    for (int e = threadIdx.x; e < K; e += blockDim.x) sg[e] = gld(s.g + e);
    __syncthreads();
    if (s.N <= kGroupMaxN)
      loewner_body<kSmallGroup, true>(s.counts, sg, s.rho, s.org, s.tau, s.what, s.status,
                                      b * (256 / kSmallGroup) + t / kSmallGroup);
    else
      loewner_body<64, true>(s.counts, sg, s.rho, s.org, s.tau, s.what, s.status, b * 4 + (t >> 6));
  } else {
    loewner_body<64, false>(s.counts, s.g, s.rho, s.org, s.tau, s.what, s.status, b * 4 + (t >> 6));
  }
}

// Block shapes and the LDS copy of the poles and weights as in the secular kernel.
template <int BT>
__global__ __launch_bounds__(BT) void colnorm_kernel(StageLevel L) {
  constexpr int CAP = BT == 1024 ? kSecLdsN : kGroupMaxN;
  __shared__ double sm[2 * CAP];   // poles, then weights
  const int* boff = BT == 1024 ? L.boff_s : L.boff_i;
  const int j = find_job(boff, L.n, blockIdx.x);
  const Stage s = L.st[j];
  const int b = (blockIdx.x - boff[j]) * (BT / 256) + (threadIdx.x >> 8), t = threadIdx.x & 255;
  if (s.N <= CAP) {
    const int K = min(max(*s.counts, 0), s.N);
    for (int e = threadIdx.x; e < K; e += blockDim.x) {
      sm[e] = gld(s.g + e);
      sm[CAP + e] = gld(s.what + e);
    }
    __syncthreads();
    if (s.N <= kGroupMaxN)
      colnorm_body<kSmallGroup, true>(s.counts, sm, sm + CAP, s.org, s.tau, s.cs, s.mu, s.status,
                                      b * (256 / kSmallGroup) + t / kSmallGroup);
    else
      colnorm_body<64, true>(s.counts, sm, sm + CAP, s.org, s.tau, s.cs, s.mu, s.status, b * 4 + (t >> 6));
  } else {
    colnorm_body<64, false>(s.counts, s.g, s.what, s.org, s.tau, s.cs, s.mu, s.status, b * 4 + (t >> 6));
  }
}

__global__ __launch_bounds__(256) void merge_kernel(StageLevel L) {
  const int j = find_job(L.boff_t, L.n, blockIdx.x);
  const Stage s = L.st[j];
  merge_body(s, (blockIdx.x - L.boff_t[j]) * 256 + threadIdx.x);
}

void launch_secular_level(const StageLevel& L, int maxit, int far_field, hipStream_t st) {
  if (L.blocks_i <= 0) return;
  // far_field 1: the far-field form above kGroupMaxN; 2: at every order
  if (far_field == 2 || (far_field == 1 && L.nmax > kGroupMaxN)) {
    const int direct_max = far_field == 2 ? 0 : kGroupMaxN;
    hipLaunchKernelGGL(secular_ff_kernel, dim3(L.blocks_l), dim3(kSfThreads), 0, st, L, maxit, direct_max);
    return;
  }
  if (L.nmax <= kGroupMaxN)
    hipLaunchKernelGGL(secular_kernel<256>, dim3(L.blocks_i), dim3(256), 0, st, L, maxit);
  else
    hipLaunchKernelGGL(secular_kernel<1024>, dim3(L.blocks_s), dim3(1024), 0, st, L, maxit);
}

void launch_stage_level(const StageLevel& L, int maxit, int far_field, hipStream_t st) {
  if (L.n <= 0 || L.blocks_w <= 0) return;
  hipLaunchKernelGGL(deflate_kernel, dim3(L.n), dim3(kDeflThreads), 0, st, L);
  launch_secular_level(L, maxit, far_field, st);
  if (L.nmax <= kGroupMaxN)
    hipLaunchKernelGGL(loewner_kernel<256>, dim3(L.blocks_i), dim3(256), 0, st, L);
  else
    hipLaunchKernelGGL(loewner_kernel<1024>, dim3(L.blocks_s), dim3(1024), 0, st, L);
  if (L.nmax <= kGroupMaxN)
    hipLaunchKernelGGL(colnorm_kernel<256>, dim3(L.blocks_i), dim3(256), 0, st, L);
  else
    hipLaunchKernelGGL(colnorm_kernel<1024>, dim3(L.blocks_s), dim3(1024), 0, st, L);
  hipLaunchKernelGGL(merge_kernel, dim3(L.blocks_t), dim3(256), 0, st, L);
}

}  // namespace svdu
