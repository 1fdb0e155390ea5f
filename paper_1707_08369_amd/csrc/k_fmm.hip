// The product X C~ through the 1-D fast multipole method (Section 5 and
// Appendix D of the paper), batched over all R rows of X.
//
// For every row r the live columns of X C~ are a Cauchy sum
//   Y[r, c] = s_c f_r(mu_c),  f_r(y) = sum_k B[r, k] / (g_k - y),
// over the K merged poles g_k with charges B[r, k] = sum_{j in group k}
// zeta_j X[r, j], evaluated at the K roots mu_c. All expansion operators
// depend on the geometry only, so they are shared by the R rows and every
// step below is a row-batched small matrix product (rows contiguous in memory).
//
// Tree: count-balanced over the sorted poles (leaf size s ~ 2p, Appendix D
// Step 2); root i sits in the leaf of pole i (the roots interlace the poles).
// Box intervals cover the box's poles and roots. Far field: the Chebyshev
// interpolation of Appendix D (nodes t_i = cos((2i-1) pi / 2p), Lagrange
// basis u_j, Steps 3-4) applied with each box's own centre and radius, which
// is what an adaptive tree needs (uniform levels fail on spectra spanning many
// decades):
//   P2M  W_k = sum_j B_j u_k((g_j - c)/r)                  (anterpolation)
//   M2M  W^P_k += sum_k' W^C_k' u_k((x^C_k' - c_P)/r_P)
//   M2L  L^T_k += sum_k' W^S_k' / (x^S_k' - y^T_k)
//   L2L  L^C_k += sum_k' L^P_k' u_k'((y^C_k - c_P)/r_P)
//   L2P  f_far(y) = sum_k L^T_k u_k((y - c_T)/r_T)
// Two boxes interact through M2L when the gap between their intervals is at
// least the larger of their widths, so every interpolation sees its nearest
// singularity at >= 3 radii (error ~ (3 + sqrt 8)^-p per interpolation).
// Leaf pairs that never become admissible are summed directly (P2P) with the
// pole-relative differences (g_k - d_org) - tau of the direct path.
// Points that would stretch a box across a gap stay out of the intervals: the
// extreme root outside the pole range, an extreme pole far from the others
// (applied to every root directly) and the root in its gap; those roots are
// evaluated on their own, from the expansions of the boxes admissible for them
// plus their near leaves exactly (M2P + P2P).
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "device_util.h"
#include "fmm_plan.h"
#include "svdu_internal.h"

namespace svdu {

constexpr int kP = kFmmMaxOrder;  // padded expansion length (p <= 16)

// The host tree (box intervals, interaction lists) is built in fmm_tree.h.

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
struct FmmDev {
  int p, s, K, nlev, nbox, R;
  int droot[2];   // roots evaluated directly (-1: none)
  int ndroot;     // how many (the first ndroot entries)
  int opole;      // pole applied to every root directly (-1: none)
  int dm2p_ptr[3], dp2p_ptr[3];
  const int* dm2p;   // per direct root: boxes taken from their multipole coefficients
  const int* dp2p;   // per direct root: leaves summed exactly
  const double* lo;
  const double* hi;
  const int* s0;
  const int* s1;
  const int* m2l_ptr;
  const int* m2l_src;
  const int* near_ptr;
  const int* near_src;
  const double* cheb;   // ChebTab of order p (kChebWords doubles)
  double* B;   // [K][R] charges
  double* W;   // [nbox][kP][R] far-field coefficients
  double* L;   // [nbox][kP][R] local coefficients
};

// Chebyshev nodes t_k (Appendix D Step 3) and the inverse node differences
// 1/(t_k - t_m), built once per plan on the host (cheb_table) and copied into
// LDS by every block; then each Lagrange basis value
// u_k(t) = prod_{m != k} (t - t_m) / (t_k - t_m) (Step 4) costs p multiplies.
struct ChebTab {
  double t[kP];
  double inv[kP * kP];
};
constexpr int kChebWords = kP + kP * kP;

__device__ __forceinline__ void cheb_fill(ChebTab* T, const FmmDev& F) {
  double* dst = T->t;   // t and inv are contiguous
  for (int e = threadIdx.x; e < kChebWords; e += blockDim.x) dst[e] = gld(F.cheb + e);
}

__device__ __forceinline__ double lagrange(const ChebTab& T, int k, int p, double x) {
  double v = 1.0;
  for (int m = 0; m < p; ++m)
    if (m != k) v *= (x - T.t[m]) * T.inv[k * kP + m];
  return v;
}

__device__ __forceinline__ void box_cr(const FmmDev& F, int id, double* c, double* r) {
  const double lo = F.lo[id], hi = F.hi[id];
  *c = 0.5 * (lo + hi);
  *r = fmax(0.5 * (hi - lo), fmax(fabs(*c) * 1e-14, 1e-300));
}

// ---------------------------------------------------------------------------
// Wide groups (more than kWideGroup members; with n > m the exact zero block
// of the right-hand eigen-updates is one): sum_{q in group} w_j X[r, j] for the
// rows r0 + 32 u + tid / 8 (u < NSUB) by a whole 256-thread block. The
// members' columns and weights go through LDS in rounds of kGroupChunk; the 8
// threads of a row add every eighth member and are summed in a fixed order.
// Called by the whole block; every thread of a row receives its sum.
// ---------------------------------------------------------------------------
constexpr int kWideGroup = 64;
constexpr int kGroupChunk = 1024;
struct GroupStage {
  int col[kGroupChunk];
  double w[kGroupChunk];
};

template <int NSUB>
__device__ void wide_group_rows(const double* X, int ldx, int R, int r0, const Stage& s, int f, int sz,
                                const double* wt, GroupStage& gs, double (&acc)[NSUB]) {
  const int rr = threadIdx.x >> 3, p = threadIdx.x & 7;
#pragma unroll
  for (int u = 0; u < NSUB; ++u) acc[u] = 0.0;
  for (int m0 = 0; m0 < sz; m0 += kGroupChunk) {
    const int n = min(kGroupChunk, sz - m0);
    __syncthreads();   // the previous round is read
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const int j = gld(s.col_of + gld(s.Llist + f + m0 + e));
      gs.col[e] = j;
      gs.w[e] = gld(wt + j);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NSUB; ++u) {
      const int r = r0 + 32 * u + rr;
      if (r < R) {
        const double* xr = X + (size_t)r * ldx;
        double a = acc[u];
        for (int e = p; e < n; e += 8) a += gs.w[e] * gld(xr + gs.col[e]);
        acc[u] = a;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NSUB; ++u) {
    double a = acc[u];
    a += __shfl_xor(a, 1, 64);
    a += __shfl_xor(a, 2, 64);
    a += __shfl_xor(a, 4, 64);
    acc[u] = a;
  }
}

// ---------------------------------------------------------------------------
// charges B[k][r] = sum_{j in group k} zeta_j X[r, j]  (transpose through LDS)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fmm_charges(int R, const double* __restrict__ X, int ldx, Stage s,
                                                   double* __restrict__ B) {
  __shared__ double tile[32][33];
  __shared__ int nwide, widek[32];
  __shared__ GroupStage gs;
  if (*s.status & kStFatal) return;
  const int K = s.counts[0];
  const int k0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  if (threadIdx.x == 0) nwide = 0;
  __syncthreads();
  // the group of charge k (the same for all 32 rows): one member, or several
  // exactly equal poles; wide groups are left to the whole block below
  const int k = k0 + tx;
  int f = 0, sz = 0, j1 = 0;
  double z1 = 0.0;
  if (k < K) {
    f = gld(s.cfirst + k);
    sz = gld(s.csize + k);
    j1 = gld(s.col_of + gld(s.Llist + f));
    z1 = gld(s.rzeta + j1);
  }
  const bool wide = k < K && sz > kWideGroup;
  if (ty == 0 && wide) widek[atomicAdd(&nwide, 1)] = tx;
  for (int rr = ty; rr < 32; rr += 8) {
    const int r = r0 + rr;
    double v = 0.0;
    if (r < R && k < K && !wide) {
      if (sz == 1) {
        v += z1 * gld(X + (size_t)r * ldx + j1);
      } else {
        for (int q = f; q < f + sz; ++q) {
          const int j = gld(s.col_of + gld(s.Llist + q));
          v += gld(s.rzeta + j) * gld(X + (size_t)r * ldx + j);
        }
      }
    }
    tile[rr][tx] = v;
  }
  __syncthreads();
  for (int q = 0; q < nwide; ++q) {
    const int kx = widek[q], kk = k0 + kx;
    double acc[1];
    wide_group_rows<1>(X, ldx, R, r0, s, gld(s.cfirst + kk), gld(s.csize + kk), s.rzeta, gs, acc);
    if ((threadIdx.x & 7) == 0) tile[threadIdx.x >> 3][kx] = acc[0];
  }
  __syncthreads();
  for (int kk = ty; kk < 32; kk += 8) {
    const int k = k0 + kk, r = r0 + tx;
    if (k < K && r < R) B[(size_t)k * R + r] = tile[tx][kk];
  }
}

// ---------------------------------------------------------------------------
// Row-batched operator products on the matrix cores. Every translation of
// the expansion applies small operators (at most 32 x 32, built in LDS from
// the box geometry) to the same coefficients of all R rows:
//   out[i][r] = sum_k Op[i][k] src[k][r],
// one v_mfma_f64_16x16x4f64 per 16 operator rows, 4 k and 16 rows, with the
// operator as the A operand (lane l: Op[l % 16][k0 + l / 16]) and 16
// consecutive rows of the coefficients as B (lane l: src[k0 + l / 16][r0 +
// l % 16]); result register v of lane l holds out[l / 16 + 4 v][r0 + l % 16].
// A block builds the operators of its box once and then walks a chunk of
// rows, 256 at a time (4 waves x kNT tiles of 16 rows); all loads of an
// operator's coefficients are issued before its MFMAs.
// ---------------------------------------------------------------------------
typedef double fd4 __attribute__((ext_vector_type(4)));
constexpr int kNT = 4;                     // row tiles of 16 per wave
constexpr int kRowsPerBlock = 4 * 16 * kNT;
constexpr int kOpLd = kP + 1;              // LDS row stride of a p x p operator (odd: no bank conflicts)
#ifndef DOWN_ROW_GROUPS
#define DOWN_ROW_GROUPS 4
#endif
constexpr int kDownRowGroups = DOWN_ROW_GROUPS;   // most 256-row groups per block in the downward pass
constexpr int kS = 32;                     // largest leaf
constexpr int kLNT = 4;                    // row tiles of 16 per wave in the leaf kernel
constexpr int kLeafRows = 4 * 16 * kLNT;

template <int NT>
__device__ __forceinline__ void zero_acc(fd4 (&acc)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = fd4{0.0, 0.0, 0.0, 0.0};
}

// Coefficients src[k][rows of the wave's tiles] for k < 4 KS, zero for k >= kvalid or r >= R.
// Branch-free: every k-step is loaded (rows clamped into range, then zeroed).
template <int KS, int NT>
__device__ __forceinline__ void load_b(double (&b)[KS][NT], int kvalid, const double* src, int R, int r0) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = 4 * ks + kq;
    const bool kok = k < kvalid;
    const double* row = src + (size_t)(kok ? k : 0) * R;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int r = r0 + 16 * t + i;
      const double v = gld(row + (r < R ? r : R - 1));
      b[ks][t] = (kok && r < R) ? v : 0.0;
    }
  }
}

// acc[t] += Op[16 rows][0 .. 4 ksteps) x b[.][t]. Every k-step is issued, those
// past ksteps with a zero operator entry (b is zero there too), so the MFMA
// chain has no branches and its accumulators stay in place; op must be
// readable for all 4 KS columns.
template <int KS, int NT>
__device__ __forceinline__ void mfma_b(const double* op, int ld, int ksteps, const double (&b)[KS][NT],
                                       fd4 (&acc)[NT]) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const double av = op[i * ld + 4 * ks + kq];
    const double a = (ks < ksteps) ? av : 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[ks][t], acc[t], 0, 0, 0);
  }
}

// dst[m][r] = acc for operator rows m < mvalid (dst row stride R).
template <int NT>
__device__ __forceinline__ void store_rows(const fd4 (&acc)[NT], double* dst, int mvalid, int R, int r0) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = r0 + 16 * t + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int mi = (lane >> 4) + 4 * v;
      if (mi < mvalid && r < R) gst(dst + (size_t)mi * R + r, acc[t][v]);
    }
  }
}

// Row range of this block: chunks of whole groups of `rows` rows.
__device__ __forceinline__ void row_chunk(int R, int rows, int* rbeg, int* rend) {
  const int groups = (R + rows - 1) / rows;
  const int per = (groups + gridDim.y - 1) / gridDim.y;
  *rbeg = blockIdx.y * per * rows;
  *rend = min(R, *rbeg + per * rows);
}

// ---------------------------------------------------------------------------
// P2M on the leaves: W[leaf][kk][r] = sum_{j in leaf} u_kk((g_j - c)/rad) B[j][r]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void fmm_p2m(FmmDev F, const double* __restrict__ g, const int* status) {
  constexpr int ld = kS + 1;
  __shared__ double op[16 * ld];   // [kk][source in leaf]
  __shared__ ChebTab T;
  if (*status & kStFatal) return;
  const int id = fmm_box_id(F.nlev, blockIdx.x);
  const int a0 = F.s0[id], a1 = F.s1[id];
  if (a1 <= a0) return;
  double c, rad;
  box_cr(F, id, &c, &rad);
  const int ns = a1 - a0;
  cheb_fill(&T, F);
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * kS; e += blockDim.x) {
    const int kk = e / kS, j = e % kS;
    op[kk * ld + j] = (kk < F.p && j < ns && a0 + j != F.opole) ? lagrange(T, kk, F.p, (g[a0 + j] - c) / rad) : 0.0;
  }
  __syncthreads();
  int rbeg, rend;
  row_chunk(F.R, kRowsPerBlock, &rbeg, &rend);
  const int ksteps = (ns + 3) / 4;
  for (int rt = rbeg; rt < rend; rt += kRowsPerBlock) {
    const int r0 = rt + (threadIdx.x >> 6) * 16 * kNT;
    double b[kS / 4][kNT];
    load_b(b, ns, F.B + (size_t)a0 * F.R, F.R, r0);
    fd4 acc[kNT];
    zero_acc(acc);
    mfma_b(op, ld, ksteps, b, acc);
    store_rows(acc, F.W + (size_t)id * kP * F.R, F.p, F.R, r0);
  }
}

// ---------------------------------------------------------------------------
// M2M for one level: W[parent][kp][r] = sum_children sum_kc M[kp][kc] W[child][kc][r]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void fmm_m2m(FmmDev F, int level, const int* status) {
  __shared__ double op[2][16 * kOpLd];   // [child][kp][kc]
  __shared__ int has[2];
  __shared__ ChebTab T;
  if (*status & kStFatal) return;
  const int id = fmm_box_id(level, blockIdx.x);
  if (F.s1[id] <= F.s0[id]) return;
  double cp, rp;
  box_cr(F, id, &cp, &rp);
  const int ch[2] = {fmm_box_id(level + 1, 2 * blockIdx.x), fmm_box_id(level + 1, 2 * blockIdx.x + 1)};
  if (threadIdx.x < 2) has[threadIdx.x] = F.s1[ch[threadIdx.x]] > F.s0[ch[threadIdx.x]];
  cheb_fill(&T, F);
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * 16 * 16; e += blockDim.x) {
    const int q = e >> 8, rem = e & 255, kp = rem >> 4, kc = rem & 15;
    double v = 0.0;
    if (kp < F.p && kc < F.p && has[q]) {
      double cc, rc;
      box_cr(F, ch[q], &cc, &rc);
      v = lagrange(T, kp, F.p, (cc + rc * T.t[kc] - cp) / rp);
    }
    op[q][kp * kOpLd + kc] = v;
  }
  __syncthreads();
  int rbeg, rend;
  row_chunk(F.R, kRowsPerBlock, &rbeg, &rend);
  const int ksteps = (F.p + 3) / 4;
  for (int rt = rbeg; rt < rend; rt += kRowsPerBlock) {
    const int r0 = rt + (threadIdx.x >> 6) * 16 * kNT;
    fd4 acc[kNT];
    zero_acc(acc);
    for (int q = 0; q < 2; ++q) {
      if (!has[q]) continue;
      double b[kP / 4][kNT];
      load_b(b, F.p, F.W + (size_t)ch[q] * kP * F.R, F.R, r0);
      mfma_b(op[q], kOpLd, ksteps, b, acc);
    }
    store_rows(acc, F.W + (size_t)id * kP * F.R, F.p, F.R, r0);
  }
}

// ---------------------------------------------------------------------------
// Downward pass for one level: L[T] = L2L(L[parent]) + sum_S M2L(W[S]).
// The block lays its box's operators (L2L first, then the M2L list) side by
// side in one LDS table, p rows by 16 columns each, notes the source rows of
// every k-step, and runs one k-loop over them, one operator per chunk, with
// the loads of the next operator in flight while the current one is on the
// matrix cores. An odd operator count is padded with a zero operator on
// valid rows; more than kDownOps operators take further passes. Blocks are
// (box, group of row groups) pairs in the XCD-aware order of the leaf kernel.
// ---------------------------------------------------------------------------
constexpr int kDownOps = 8;                  // operators per pass
constexpr int kDownLd = 16 * kDownOps + 1;   // table row stride (odd)

template <int NT>
__device__ __forceinline__ void down_load(double (&b)[4][NT], int c, const double* const* ksrc, const int* kcnt,
                                          int R, int r0) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * c + ks;
    const double* row = ksrc[k] + (size_t)min(kq, kcnt[k] - 1) * R;
#pragma unroll
    for (int t = 0; t < NT; ++t) b[ks][t] = gld(row + min(r0 + 16 * t + i, R - 1));
  }
}

template <int NT>
__device__ __forceinline__ void down_mma(const double (&b)[4][NT], int c, const double* op, fd4 (&acc)[NT]) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const double a = op[i * kDownLd + 16 * c + 4 * ks + kq];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[ks][t], acc[t], 0, 0, 0);
  }
}

__global__ __launch_bounds__(256) void fmm_down(FmmDev F, int level, const int* status, int nrb, int rgpb) {
  __shared__ double op[16 * kDownLd];           // [target node][16 operator + source node]
  __shared__ const double* ksrc[4 * kDownOps];  // first source row of each k-step
  __shared__ int kcnt[4 * kDownOps];            // its valid rows (1..4)
  __shared__ double oc[kDownOps], orad[kDownOps];
  __shared__ int okind[kDownOps];               // 0 L2L, 1 M2L, -1 padding
  __shared__ int nopp;                          // operators of the pass, padded to even
  __shared__ ChebTab T;
  if (*status & kStFatal) return;
  const int nb = 1 << level, total = nb * nrb;
  const int xcd = blockIdx.x % 8, per = total / 8, extra = total % 8;
  const int w = xcd * per + min(xcd, extra) + blockIdx.x / 8;
  const int bx = w % nb, rb = w / nb;
  const int id = fmm_box_id(level, bx);
  if (F.s1[id] <= F.s0[id]) return;
  double ct, rt;
  box_cr(F, id, &ct, &rt);
  cheb_fill(&T, F);
  const int q0 = F.m2l_ptr[id], nm2l = F.m2l_ptr[id + 1] - q0;
  const int nops = (level > 0 ? 1 : 0) + nm2l;
  const int npass = max(1, (nops + kDownOps - 1) / kDownOps);
  const double* pad_src = F.W + (size_t)id * kP * F.R;   // written rows, zero weights
  auto build_pass = [&](int pass) {
    const int o0 = pass * kDownOps, cnt = max(0, min(kDownOps, nops - o0));
    const int cntp = max(2, (cnt + 1) & ~1);
    __syncthreads();   // the previous table is read by every wave
    for (int qi = threadIdx.x; qi < cntp; qi += blockDim.x) {
      const int o = o0 + qi;
      const double* src = pad_src;
      int kind = -1;
      double c = 0.0, r = 1.0;
      if (qi < cnt) {
        const bool l2l = level > 0 && o == 0;
        const int other = l2l ? fmm_box_id(level - 1, bx >> 1) : F.m2l_src[q0 + o - (level > 0 ? 1 : 0)];
        box_cr(F, other, &c, &r);
        src = (l2l ? F.L : F.W) + (size_t)other * kP * F.R;
        kind = l2l ? 0 : 1;
      }
      oc[qi] = c;
      orad[qi] = r;
      okind[qi] = kind;
      for (int j = 0; j < 4; ++j) {
        // rows >= p of W and L are never written: clamp into the first p
        ksrc[4 * qi + j] = src + (size_t)min(4 * j, F.p - 1) * F.R;
        kcnt[4 * qi + j] = max(1, min(4, F.p - 4 * j));
      }
    }
    if (threadIdx.x == 0) nopp = cntp;
    __syncthreads();
    for (int e = threadIdx.x; e < cntp * 256; e += blockDim.x) {
      const int qi = e >> 8, i = (e >> 4) & 15, k = e & 15;
      double v = 0.0;
      if (i < F.p && k < F.p && okind[qi] >= 0) {
        if (okind[qi] == 0)
          v = lagrange(T, k, F.p, (ct + rt * T.t[i] - oc[qi]) / orad[qi]);
        else
          v = 1.0 / ((oc[qi] + orad[qi] * T.t[k]) - (ct + rt * T.t[i]));
      }
      op[i * kDownLd + 16 * qi + k] = v;
    }
    __syncthreads();
  };
  if (npass == 1) build_pass(0);
  const int nrg = (F.R + kRowsPerBlock - 1) / kRowsPerBlock;
  const int rg0 = rb * rgpb, rg1 = min(rg0 + rgpb, nrg);
  for (int rg = rg0; rg < rg1; ++rg) {
    const int r0 = rg * kRowsPerBlock + (threadIdx.x >> 6) * 16 * kNT;
    fd4 acc[kNT];
    zero_acc(acc);
    for (int pass = 0; pass < npass; ++pass) {
      if (npass > 1) build_pass(pass);
      const int nch = nopp;   // even
      double bA[4][kNT], bB[4][kNT];
      down_load(bA, 0, ksrc, kcnt, F.R, r0);
      for (int c = 0; c < nch; c += 2) {
        down_load(bB, c + 1, ksrc, kcnt, F.R, r0);
        down_mma(bA, c, op, acc);
        // branch-free: the last pair reloads its own operator
        down_load(bA, min(c + 2, nch - 1), ksrc, kcnt, F.R, r0);
        down_mma(bB, c + 1, op, acc);
      }
    }
    store_rows(acc, F.L + (size_t)id * kP * F.R, F.p, F.R, r0);
  }
}

// ---------------------------------------------------------------------------
// Leaves: L2P + P2P, scaled by the column scale, written to the output
// positions of the roots. For the targets t of a leaf (at most kS = 32 roots,
// two 16-row operator blocks) both parts are one contraction,
//   Y[t][r] = sum_kk u_kk(y_t) L[leaf][kk][r]
//           + sum_{near boxes S} sum_{j in S} B[j][r] / ((g_j - d_org(t)) - tau_t),
// so the block lays the L2P weights and the near-field reciprocals side by
// side in one LDS operator table, notes the first source row of every k-step
// of 4, and runs one k-loop in chunks of kLeafChunk k-steps: the loads of the
// next chunk are in flight while the current one is on the matrix cores. The
// k-steps keep the order of the parts (L2P, then the near list), and padding
// k-steps carry zero weights on a valid row. A near list longer than
// kLeafNearPass boxes takes further passes over the same accumulators.
// Blocks are (leaf, 256-row group) pairs in an XCD-aware order: the blocks of
// one XCD take consecutive leaves of one row group, whose near fields read the
// same charge rows, in that XCD's L2. Results go from the accumulators to the
// output directly.
// Like the translation kernels it declares no blocks-per-CU minimum: with the
// whole register file available the MFMA accumulators live in AGPRs.
// ---------------------------------------------------------------------------
constexpr int kLeafKs = 48;                  // k-steps of 4 in the operator table
constexpr int kLeafLd = 4 * kLeafKs + 1;     // its row stride in doubles (odd: conflict-free reads)
constexpr int kLeafChunk = 4;                // k-steps per pipelined chunk
constexpr int kLeafNearPass = 5;             // near boxes per pass: 4 + 5 * 8 <= kLeafKs k-steps
#ifndef LEAF_ROW_GROUPS
#define LEAF_ROW_GROUPS 4
#endif
constexpr int kLeafRowGroups = LEAF_ROW_GROUPS;   // 256-row groups per block (one table build each)
static_assert(4 + 1 + kLeafNearPass * (kS / 4) <= kLeafKs, "a pass must fit the operator table");
static_assert(kLeafKs % (2 * kLeafChunk) == 0, "the table holds whole chunk pairs");

template <int NT>
__device__ __forceinline__ void leaf_load(double (&b)[kLeafChunk][NT], int c, const double* const* ksrc,
                                          const int* kcnt, int R, int r0) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < kLeafChunk; ++ks) {
    const int k = c * kLeafChunk + ks;
    const double* row = ksrc[k] + (size_t)min(kq, kcnt[k] - 1) * R;
#pragma unroll
    for (int t = 0; t < NT; ++t) b[ks][t] = gld(row + min(r0 + 16 * t + i, R - 1));
  }
}

template <int NT>
__device__ __forceinline__ void leaf_mma(const double (&b)[kLeafChunk][NT], int c, const double* op, fd4 (&acc0)[NT],
                                         fd4 (&acc1)[NT]) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < kLeafChunk; ++ks) {
    const int col = 4 * (c * kLeafChunk + ks) + kq;
    const double a0 = op[i * kLeafLd + col], a1 = op[(16 + i) * kLeafLd + col];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc0[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b[ks][t], acc0[t], 0, 0, 0);
      acc1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b[ks][t], acc1[t], 0, 0, 0);
    }
  }
}

__global__ __launch_bounds__(256) void fmm_leaf_eval(FmmDev F, Stage s, double* __restrict__ Xo, int ldo,
                                                      const double* __restrict__ colscale, int nrb, int rgpb) {
  __shared__ double op[kS * kLeafLd];          // [target][column = 4 k-step + kq]
  __shared__ const double* ksrc[kLeafKs];      // first source row of each k-step
  __shared__ int kcnt[kLeafKs];                // its valid rows (1..4)
  __shared__ int kseg[kLeafKs];                // -1 L2P, -3 isolated pole, q near box q of the pass, -2 padding
  __shared__ double colg[4 * kLeafKs];         // source pole of each near-field column
  __shared__ int nb0[kLeafNearPass], nns[kLeafNearPass], nks0[kLeafNearPass + 1];
  __shared__ int pos[kS];
  __shared__ double scl[kS], tgo[kS], tgt[kS];
  __shared__ ChebTab T;
  if (*s.status & kStFatal) return;
  // blocks with equal index mod 8 share an XCD: give them consecutive work
  const int nleaf = 1 << F.nlev, total = nleaf * nrb;
  const int xcd = blockIdx.x % 8, per = total / 8, extra = total % 8;
  const int w = xcd * per + min(xcd, extra) + blockIdx.x / 8;
  const int leaf = w % nleaf, rb = w / nleaf;
  const int id = fmm_box_id(F.nlev, leaf);
  const int a0 = F.s0[id], a1 = F.s1[id];
  if (a1 <= a0) return;
  const int nt = a1 - a0;
  double ct, rt;
  box_cr(F, id, &ct, &rt);
  cheb_fill(&T, F);
  const int q0 = F.near_ptr[id], nnear = F.near_ptr[id + 1] - q0;
  // per target: origin pole, offset, column position and scale (one load each)
  for (int t = threadIdx.x; t < kS; t += blockDim.x) {
    const int i = a0 + t;
    int P = -1;
    double sc = 0.0, go = 0.0, ta = 0.0;
    if (t < nt) {
      P = gld(s.rootpos + i);
      sc = (colscale ? gld(colscale + P) : 1.0) * gld(s.cs + i);
      go = gld(s.g + gld(s.org + i));
      ta = gld(s.tau + i);
      if (i == F.droot[0] || i == F.droot[1]) P = -1;   // evaluated by fmm_direct_roots
    }
    pos[t] = P;
    scl[t] = sc;
    tgo[t] = go;
    tgt[t] = ta;
  }
  const int lane = threadIdx.x & 63, kq = lane >> 4;
  const double* Lsrc = F.L + (size_t)id * kP * F.R;
  const int npass = max(1, (nnear + kLeafNearPass - 1) / kLeafNearPass);
  // operator table of one pass (all threads; starts and ends with a barrier)
  auto build_pass = [&](int pass) {
    const int qa = pass * kLeafNearPass, nq = min(kLeafNearPass, nnear - qa);
    __syncthreads();   // the previous table is read by every wave
    if ((int)threadIdx.x < nq) {
      const int nbx = F.near_src[q0 + qa + threadIdx.x];
      nb0[threadIdx.x] = F.s0[nbx];
      nns[threadIdx.x] = F.s1[nbx] - F.s0[nbx];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      // the first pass starts with the 4 L2P k-steps and the isolated pole's
      int k = (pass == 0) ? 4 + (F.opole >= 0 ? 1 : 0) : 0;
      for (int q = 0; q < nq; ++q) {
        nks0[q] = k;
        k += (nns[q] + 3) / 4;
      }
      nks0[nq] = k;
      nks0[kLeafNearPass] = k;       // the pass's k-step count, for readers that do not know nq
    }
    __syncthreads();
    const int nks = nks0[nq];
    const int nksp = (nks + 2 * kLeafChunk - 1) / (2 * kLeafChunk) * (2 * kLeafChunk);
    for (int k = threadIdx.x; k < nksp; k += blockDim.x) {
      const double* src = Lsrc;   // padding: zero weights on a written row of L
      int cnt = 1, seg = -2;
      if (k < nks) {
        if (pass == 0 && k < 4) {
          // rows kk >= p of L are never written: clamp into the first p
          src = Lsrc + (size_t)min(4 * k, F.p - 1) * F.R;
          cnt = max(1, min(4, F.p - 4 * k));
          seg = -1;
        } else if (pass == 0 && k == 4 && F.opole >= 0) {
          src = F.B + (size_t)F.opole * F.R;
          seg = -3;
          for (int e = 0; e < 4; ++e) colg[4 * k + e] = e == 0 ? gld(s.g + F.opole) : 0.0;
        } else {
          int q = 0;
          while (q + 1 < nq && k >= nks0[q + 1]) ++q;
          const int j0 = 4 * (k - nks0[q]);
          src = F.B + (size_t)(nb0[q] + j0) * F.R;
          cnt = min(4, nns[q] - j0);
          seg = q;
          for (int e = 0; e < 4; ++e) colg[4 * k + e] = (j0 + e < nns[q]) ? gld(s.g + nb0[q] + j0 + e) : 0.0;
        }
      }
      ksrc[k] = src;
      kcnt[k] = cnt;
      kseg[k] = seg;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kS * 4 * nksp; e += blockDim.x) {
      const int t = e & (kS - 1), col = e / kS, k = col >> 2;
      const int seg = kseg[k];
      double v = 0.0;
      if (t < nt && pos[t] >= 0) {
        if (seg == -1) {
          if (col < F.p) v = lagrange(T, col, F.p, ((tgo[t] + tgt[t]) - ct) / rt);
        } else if (seg == -3) {
          if ((col & 3) == 0) v = 1.0 / ((colg[col] - tgo[t]) - tgt[t]);
        } else if (seg >= 0) {
          const int j = 4 * (k - nks0[seg]) + (col & 3);
          if (j < nns[seg] && nb0[seg] + j != F.opole) v = 1.0 / ((colg[col] - tgo[t]) - tgt[t]);
        }
      }
      op[t * kLeafLd + col] = v;
    }
    __syncthreads();
  };
  __syncthreads();   // pos, scl, tgo, tgt are read by every wave from here on
  if (npass == 1) build_pass(0);
  // lane l holds targets l / 16 + 4 v (acc0) and 16 + l / 16 + 4 v (acc1) of rows r0 + 16 t + l % 16
  int P0[4], P1[4];
  double S0[4], S1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    P0[v] = pos[kq + 4 * v];
    S0[v] = scl[kq + 4 * v];
    P1[v] = pos[16 + kq + 4 * v];
    S1[v] = scl[16 + kq + 4 * v];
  }
  const int rg0 = rb * rgpb, rg1 = min(rg0 + rgpb, (F.R + kLeafRows - 1) / kLeafRows);
  for (int rg = rg0; rg < rg1; ++rg) {
    const int r0 = rg * kLeafRows + (threadIdx.x >> 6) * 16 * kLNT;
    fd4 acc0[kLNT], acc1[kLNT];
    zero_acc(acc0);
    zero_acc(acc1);
    for (int pass = 0; pass < npass; ++pass) {
      if (npass > 1) build_pass(pass);
      const int nks = nks0[kLeafNearPass];
      const int nch = (nks + 2 * kLeafChunk - 1) / (2 * kLeafChunk) * 2;   // even
      double bA[kLeafChunk][kLNT], bB[kLeafChunk][kLNT];
      leaf_load(bA, 0, ksrc, kcnt, F.R, r0);
      for (int c = 0; c < nch; c += 2) {
        leaf_load(bB, c + 1, ksrc, kcnt, F.R, r0);
        leaf_mma(bA, c, op, acc0, acc1);
        // branch-free: the last pair reloads its own chunk, so the accumulators stay in place
        leaf_load(bA, min(c + 2, nch - 1), ksrc, kcnt, F.R, r0);
        leaf_mma(bB, c + 1, op, acc0, acc1);
      }
    }
#pragma unroll
    for (int t = 0; t < kLNT; ++t) {
      const int row = r0 + 16 * t + (lane & 15);
      if (row < F.R) {
        double* o = Xo + (size_t)row * ldo;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (P0[v] >= 0) gst(o + P0[v], S0[v] * acc0[t][v]);
          if (P1[v] >= 0) gst(o + P1[v], S1[v] * acc1[t][v]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The roots evaluated directly (at most two, F.droot): for a root y at
// d_org + tau, the far field from the multipole coefficients of the boxes
// listed for it, f(y) = sum_k W_k / (x_k - y) over each box's Chebyshev nodes,
// the listed leaves exactly with pole-relative differences (g_j - d_org) - tau,
// and the isolated pole, summed in that order and scaled by the column scale.
// Terms go through LDS in rounds of kDirTerms (weight and source row); a block
// takes 64 rows, and its four waves add every fourth term of a round for
// them, summed in a fixed order at the end.
// ---------------------------------------------------------------------------
constexpr int kDirTerms = 512;

__global__ __launch_bounds__(256) void fmm_direct_roots(FmmDev F, Stage s, double* __restrict__ Xo, int ldo,
                                                        const double* __restrict__ colscale) {
  __shared__ double wt[kDirTerms];
  __shared__ const double* src[kDirTerms];
  __shared__ double part[4][64];
  __shared__ ChebTab T;
  if (*s.status & kStFatal) return;
  const int d = blockIdx.y, i = F.droot[d];
  const double go = gld(s.g + gld(s.org + i)), ta = gld(s.tau + i), y = go + ta;
  const int m0 = F.dm2p_ptr[d], nm = F.dm2p_ptr[d + 1] - m0;
  const int p0 = F.dp2p_ptr[d], np = F.dp2p_ptr[d + 1] - p0;
  // term t: far (box m0 + t / kP, node t % kP), near (leaf p0 + u / kS, pole u % kS), then the isolated pole
  const int nfar = nm * kP, nterm = nfar + np * kS + (F.opole >= 0 ? 1 : 0);
  cheb_fill(&T, F);
  const int ph = threadIdx.x >> 6, r = blockIdx.x * 64 + (threadIdx.x & 63);
  double acc = 0.0;
  for (int t0 = 0; t0 < nterm; t0 += kDirTerms) {
    __syncthreads();   // T is written, and the previous round is read
    for (int e = threadIdx.x; e < kDirTerms && t0 + e < nterm; e += blockDim.x) {
      const int t = t0 + e;
      double w = 0.0;
      const double* sr = F.B;   // zero weights point at row 0 of the charges
      if (t < nfar) {
        const int bx = F.dm2p[m0 + t / kP], kk = t % kP;
        double c, rad;
        box_cr(F, bx, &c, &rad);
        // rows kk >= p of W are never written
        sr = F.W + ((size_t)bx * kP + min(kk, F.p - 1)) * F.R;
        if (kk < F.p) w = 1.0 / ((c + rad * T.t[kk]) - y);
      } else if (t < nfar + np * kS) {
        const int u = t - nfar, lf = F.dp2p[p0 + u / kS], j = F.s0[lf] + u % kS;
        if (j < F.s1[lf] && j != F.opole) {
          sr = F.B + (size_t)j * F.R;
          w = 1.0 / ((gld(s.g + j) - go) - ta);
        }
      } else {
        sr = F.B + (size_t)F.opole * F.R;
        w = 1.0 / ((gld(s.g + F.opole) - go) - ta);
      }
      wt[e] = w;
      src[e] = sr;
    }
    __syncthreads();
    const int ne = min(kDirTerms, nterm - t0);
    if (r < F.R) {
#pragma unroll 8
      for (int e = ph; e < ne; e += 4) acc += wt[e] * gld(src[e] + r);
    }
  }
  part[ph][threadIdx.x & 63] = acc;
  __syncthreads();
  if (ph == 0 && r < F.R) {
    const int l = threadIdx.x;
    const int P = gld(s.rootpos + i);
    const double sc = (colscale ? gld(colscale + P) : 1.0) * gld(s.cs + i);
    gst(Xo + (size_t)r * ldo + P, sc * (((part[0][l] + part[1][l]) + part[2][l]) + part[3][l]));
  }
}

// ---------------------------------------------------------------------------
// Deflated output columns: Xo[r, c] = X[r, mem] - 2 h_c sum_{j in group} rh_j X[r, j]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fmm_group_dots(int R, const double* __restrict__ X, int ldx, Stage s,
                                                      double* __restrict__ hX) {
  __shared__ GroupStage gs;
  if (*s.status & kStFatal) return;
  const int c = blockIdx.x;
  const int K = s.counts[0];
  if (c >= K || s.csize[c] < 2) return;
  const int f = s.cfirst[c], sz = s.csize[c];
  if (sz > kWideGroup) {   // the block's 256 rows together
    double acc[8];
    const int r0 = blockIdx.y * blockDim.x;
    wide_group_rows<8>(X, ldx, R, r0, s, f, sz, s.rh, gs, acc);
    if ((threadIdx.x & 7) == 0)
      for (int u = 0; u < 8; ++u) {
        const int r = r0 + 32 * u + (threadIdx.x >> 3);
        if (r < R) hX[(size_t)c * R + r] = acc[u];
      }
    return;
  }
  const int r = blockIdx.y * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double a = 0.0;
  for (int q = f; q < f + sz; ++q) {
    const int j = s.col_of[s.Llist[q]];
    a += s.rh[j] * X[(size_t)r * ldx + j];
  }
  hX[(size_t)c * R + r] = a;
}

// Block: 32 deflated columns (consecutive output and source columns for a
// merged group) x 8 rows, so that loads and stores run along the rows.
__global__ __launch_bounds__(256) void fmm_deflated_cols(int R, const double* __restrict__ X, int ldx, Stage s,
                                                         const double* __restrict__ hX, double* __restrict__ Xo,
                                                         int ldo, const double* __restrict__ colscale) {
  if (*s.status & kStFatal) return;
  const int Kd = s.counts[1], K = s.counts[0];
  const int kd = blockIdx.x * 32 + (threadIdx.x & 31), r = blockIdx.y * 8 + (threadIdx.x >> 5);
  if (kd >= Kd || r >= R) return;
  const int P = s.dpos[kd];
  const int mem = s.cmem[P], cl = s.ccl[P];
  const double h = s.ch[P];
  double v = X[(size_t)r * ldx + mem];
  if (h != 0.0 && cl >= 0 && cl < K) v -= 2.0 * h * hX[(size_t)cl * R + r];
  Xo[(size_t)r * ldo + P] = (colscale ? colscale[P] : 1.0) * v;
}

// ---------------------------------------------------------------------------
// host side: plan building, upload and launch
// ---------------------------------------------------------------------------
static size_t tree_boxes(int N) {
  int nlev = 0;   // as in fmm_build_tree: leaves of at most 32 poles
  while ((N + (1 << nlev) - 1) >> nlev > 32) ++nlev;
  return (size_t(1) << (nlev + 1)) - 1;
}

size_t fmm_workspace_elems(int R, int N) {
  // charges B (N R) + W and L (nbox kP R each) + group dot products (N R, by group id)
  return (size_t)N * R + 2 * tree_boxes(N) * kP * (size_t)R + (size_t)N * R;
}

size_t fmm_plan_bytes(int N) {
  const size_t nbox = tree_boxes(N);
  // intervals, ranges, CSR pointers, list space (<= 64 entries per box), the
  // direct roots' lists (each box at most once per root), 256-byte alignment
  return sizeof(double) * (2 * nbox + kP + kP * kP) + sizeof(int) * (4 * nbox + 2 + 2 * 64 * nbox + 4 * nbox) +
         16 * 256;
}

// Builds the plan of one product from host copies of the stage's poles g (K)
// and roots mu (K) and appends its arrays to `blob` (256-byte aligned pieces).
void fmm_prepare(int K, const double* g_host, const double* mu_host, double eps, std::vector<char>* blob,
                 FmmPrepared* out) {
  const int p = fmm_order(eps);
  if (K > 0) fmm_build_tree(K, g_host, mu_host, p, &out->P);
  out->P.p = p;
  out->P.K = K;
  const FmmHostPlan& P = out->P;
  auto add = [&](const void* src, size_t bytes) {
    size_t o = (blob->size() + 255) & ~size_t(255);
    blob->resize(o + bytes);
    if (bytes) std::memcpy(blob->data() + o, src, bytes);
    return o;
  };
  const size_t nb = P.nbox;
  out->off[0] = add(P.lo.data(), nb * sizeof(double));
  out->off[1] = add(P.hi.data(), nb * sizeof(double));
  out->off[2] = add(P.s0.data(), nb * sizeof(int));
  out->off[3] = add(P.s1.data(), nb * sizeof(int));
  out->off[4] = add(P.m2l_ptr.data(), P.m2l_ptr.size() * sizeof(int));
  out->off[5] = add(P.m2l_src.data(), P.m2l_src.size() * sizeof(int));
  out->off[6] = add(P.near_ptr.data(), P.near_ptr.size() * sizeof(int));
  out->off[7] = add(P.near_src.data(), P.near_src.size() * sizeof(int));
  out->off[8] = add(P.dm2p.data(), P.dm2p.size() * sizeof(int));
  out->off[9] = add(P.dp2p.data(), P.dp2p.size() * sizeof(int));
  // Chebyshev nodes of order p and their inverse differences (ChebTab layout)
  std::vector<double> cheb(kP + kP * kP, 0.0);
  for (int k = 0; k < p; ++k) cheb[k] = std::cos((2.0 * k + 1.0) * M_PI / (2.0 * p));
  for (int k = 0; k < p; ++k)
    for (int m = 0; m < p; ++m) cheb[kP + k * kP + m] = (k == m) ? 0.0 : 1.0 / (cheb[k] - cheb[m]);
  out->off[10] = add(cheb.data(), cheb.size() * sizeof(double));
}

// Enqueues the FMM product X_out = X C~ for stage `s` with a prepared plan
// whose arrays sit at `plan_dev` (the uploaded blob). Returns 0 or -2 when the
// workspace is too small.
int fmm_launch(int R, const double* X, int ldx, const Stage& s, const FmmPrepared& pp, const char* plan_dev,
               double* Xo, int ldo, const double* colscale, double* work, size_t work_elems, hipStream_t st) {
  const FmmHostPlan& P = pp.P;
  const int N = s.N, K = P.K;
  if (R <= 0 || N <= 0) return 0;
  const size_t nb = P.nbox;
  FmmDev F{};
  F.p = P.p;
  F.s = P.s;
  F.K = K;
  F.nlev = P.nlev;
  F.nbox = P.nbox;
  F.R = R;
  F.droot[0] = F.droot[1] = -1;
  F.ndroot = 0;
  if (P.outlier >= 0) F.droot[F.ndroot++] = P.outlier;
  if (P.outlier2 >= 0) F.droot[F.ndroot++] = P.outlier2;
  F.opole = P.opole;
  F.lo = reinterpret_cast<const double*>(plan_dev + pp.off[0]);
  F.hi = reinterpret_cast<const double*>(plan_dev + pp.off[1]);
  F.s0 = reinterpret_cast<const int*>(plan_dev + pp.off[2]);
  F.s1 = reinterpret_cast<const int*>(plan_dev + pp.off[3]);
  F.m2l_ptr = reinterpret_cast<const int*>(plan_dev + pp.off[4]);
  F.m2l_src = reinterpret_cast<const int*>(plan_dev + pp.off[5]);
  F.near_ptr = reinterpret_cast<const int*>(plan_dev + pp.off[6]);
  F.near_src = reinterpret_cast<const int*>(plan_dev + pp.off[7]);
  F.dm2p = reinterpret_cast<const int*>(plan_dev + pp.off[8]);
  F.dp2p = reinterpret_cast<const int*>(plan_dev + pp.off[9]);
  F.cheb = reinterpret_cast<const double*>(plan_dev + pp.off[10]);
  for (int d = 0; d < 3; ++d) {
    F.dm2p_ptr[d] = P.dm2p_ptr[d];
    F.dp2p_ptr[d] = P.dp2p_ptr[d];
  }
  const size_t hx_elems = (size_t)N * R;   // indexed by group id < K <= N
  if ((size_t)K * R + 2 * nb * kP * (size_t)R + hx_elems > work_elems) return -2;
  F.B = work;
  F.W = work + (size_t)K * R;
  F.L = F.W + nb * kP * (size_t)R;
  double* hX = work + (work_elems - hx_elems);
  const int rb = (R + kRowsPerBlock - 1) / kRowsPerBlock;
  // one block per (box, 256-row group): the kernels are bound by memory
  // latency, so they need every block they can get (building a box's
  // operators once per block is cheap next to that)
  auto chunks = [&](int boxes) {
    (void)boxes;
    return rb;
  };
  if (K > 0) {
    hipLaunchKernelGGL(fmm_charges, dim3((K + 31) / 32, (R + 31) / 32), dim3(256), 0, st, R, X, ldx, s, F.B);
    hipLaunchKernelGGL(fmm_p2m, dim3(1 << P.nlev, chunks(1 << P.nlev)), dim3(256), 0, st, F, s.g, s.status);
    for (int l = P.nlev - 1; l >= 0; --l)
      hipLaunchKernelGGL(fmm_m2m, dim3(1 << l, chunks(1 << l)), dim3(256), 0, st, F, l, s.status);
    for (int l = 0; l <= P.nlev; ++l) {
      // enough blocks to fill the chip, then up to kDownRowGroups row groups per block
      const int rgpb = std::max(1, std::min(kDownRowGroups, ((1 << l) * rb) / 2048));
      const int nrb = (rb + rgpb - 1) / rgpb;
      hipLaunchKernelGGL(fmm_down, dim3((1 << l) * nrb), dim3(256), 0, st, F, l, s.status, nrb, rgpb);
    }
    const int nrg = (R + kLeafRows - 1) / kLeafRows, nrb = (nrg + kLeafRowGroups - 1) / kLeafRowGroups;
    hipLaunchKernelGGL(fmm_leaf_eval, dim3((1 << P.nlev) * nrb), dim3(256), 0, st, F, s, Xo, ldo, colscale, nrb,
                       kLeafRowGroups);
    if (F.ndroot > 0)
      hipLaunchKernelGGL(fmm_direct_roots, dim3((R + 63) / 64, F.ndroot), dim3(256), 0, st, F, s, Xo, ldo, colscale);
  }
  if (K < N) {
    hipLaunchKernelGGL(fmm_group_dots, dim3(std::max(K, 1), rb), dim3(256), 0, st, R, X, ldx, s, hX);
    hipLaunchKernelGGL(fmm_deflated_cols, dim3((N - K + 31) / 32, (R + 7) / 8), dim3(256), 0, st, R, X, ldx, s, hX,
                       Xo, ldo, colscale);
  }
  return 0;
}

}  // namespace svdu
