// Products with the Cauchy eigenvector matrix C~ of one eigen-update:
// y = C~^T x for up to three vectors. It carries the projected vectors between
// the two eigen-updates of one side in core space (z for the second update is
// C~^T of the first applied to U^T b1, since U~^T b1 = C~^T U^T b1) and maps
// the sign probes.
#include "cauchy_tile.h"
#include "jobs.h"

namespace svdu {

// ---------------------------------------------------------------------------
// y = C~^T x
// ---------------------------------------------------------------------------
// Dot products of the Householder vectors of clusters of equal poles with up
// to three vectors: hx[3 c + v] = sum over members of rh_j x_v[j]. A block
// takes 256 clusters, one thread each; clusters of more than kWideDots
// members are listed and done by the whole block (fixed-order block sums).
constexpr int kWideDots = 64;

__device__ void householder_dots_member_sum(const Stage& s, int f, int e, int k0, int step, int nv,
                                            const double* x0, const double* x1, const double* x2, double* a) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = f + k0; k < e; k += step) {
    const int j = s.col_of[s.Llist[k]];
    const double h = s.rh[j];
    a0 += h * x0[j];
    if (nv > 1) a1 += h * x1[j];
    if (nv > 2) a2 += h * x2[j];
  }
  a[0] = a0;
  a[1] = a1;
  a[2] = a2;
}

// One pass of y = C~^T x over the rows of a live column, NV vectors, rows
// j0, j0 + STEP, ... in order; a zero weight adds a signed zero, which leaves
// the sum as it is. The fast pass records whether any nonzero weight met a
// |delta| below recip_fast's range; the exact pass (div_by) then repeats it
// with the same terms in the same order.
// Row poles rg and weights rz: the descriptor's arrays in global memory, or
// (LDS) the block's copy of them.
template <bool LDS>
__device__ __forceinline__ double tmv_ld(const double* p) {
  if (LDS) return *((const __attribute__((address_space(3))) double*)p);
  return gld(p);
}

template <int NV, bool EXACT, int STEP, bool LDS>
__device__ inline void tmv_pass(const CauchyDesc& d, const ColDesc& cd, const double* rg, const double* rz,
                                const double* x0, const double* x1, const double* x2, int j0, double (&acc)[3],
                                bool* tiny) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  bool t = false;
#pragma unroll 4
  for (int j = j0; j < d.N; j += STEP) {
    const double z = tmv_ld<LDS>(rz + j);
    const double del = (tmv_ld<LDS>(rg + j) - cd.o) - cd.t;
    double w;
    if (EXACT) {
      w = (z == 0.0) ? 0.0 : div_by(z, del);
    } else {
      t |= (z != 0.0) & recip_tiny(del);
      const double r = recip_fast(del);
      w = (z == 0.0) ? 0.0 : z * r;
    }
    a0 = __builtin_fma(w, gld(x0 + j), a0);
    if (NV > 1) a1 = __builtin_fma(w, gld(x1 + j), a1);
    if (NV > 2) a2 = __builtin_fma(w, gld(x2 + j), a2);
  }
  acc[0] = a0;
  acc[1] = a1;
  acc[2] = a2;
  *tiny = t;
}

// The column belongs to an aligned group of G lanes (lanes over rows, summed
// across the group afterwards).
template <int NV, int G, bool LDS>
__device__ inline void tmv_live(const CauchyDesc& d, const ColDesc& cd, const double* rg, const double* rz,
                                const double* x0, const double* x1, const double* x2, int sub, double (&acc)[3]) {
  bool tiny = false;
  tmv_pass<NV, false, G, LDS>(d, cd, rg, rz, x0, x1, x2, sub, acc, &tiny);
  if (group_any<G>(tiny)) tmv_pass<NV, true, G, LDS>(d, cd, rg, rz, x0, x1, x2, sub, acc, &tiny);
}

// Column c of y = C~^T x, for an aligned group of G lanes.
template <int G, bool LDS>
__device__ void cauchy_tmatvec_body(const CauchyDesc& d, const double* rg, const double* rz,
                                    const double* __restrict__ hx, int nv, const double* __restrict__ x0,
                                    const double* __restrict__ x1, const double* __restrict__ x2, double* y0,
                                    double* y1, double* y2, int c) {
  if (*d.status & kStFatal) return;
  const int sub = threadIdx.x & (G - 1);
  if (c >= d.N) return;
  const ColDesc cd = load_col(d, c);
  if (cd.type == 0) {
    double acc[3];
    if (nv > 2)
      tmv_live<3, G, LDS>(d, cd, rg, rz, x0, x1, x2, sub, acc);
    else if (nv > 1)
      tmv_live<2, G, LDS>(d, cd, rg, rz, x0, x1, x2, sub, acc);
    else
      tmv_live<1, G, LDS>(d, cd, rg, rz, x0, x1, x2, sub, acc);
    const double a0 = group_sum<G>(acc[0]);
    const double a1 = nv > 1 ? group_sum<G>(acc[1]) : 0.0;
    const double a2 = nv > 2 ? group_sum<G>(acc[2]) : 0.0;
    if (sub == 0) {
      y0[c] = cd.s * a0;
      if (nv > 1) y1[c] = cd.s * a1;
      if (nv > 2) y2[c] = cd.s * a2;
    }
  } else if (sub == 0 && cd.mem >= 0 && cd.mem < d.N) {
    const bool hh = cd.h != 0.0 && cd.cl >= 0 && cd.cl < d.N;
    y0[c] = x0[cd.mem] - (hh ? 2.0 * cd.h * hx[3 * cd.cl] : 0.0);
    if (nv > 1) y1[c] = x1[cd.mem] - (hh ? 2.0 * cd.h * hx[3 * cd.cl + 1] : 0.0);
    if (nv > 2) y2[c] = x2[cd.mem] - (hh ? 2.0 * cd.h * hx[3 * cd.cl + 2] : 0.0);
  }
}

// Level kernels over the jobs of a StageLevel (jobs with nv = 0 do nothing).
__global__ __launch_bounds__(256) void householder_dots(StageLevel L) {
  __shared__ int nwide, wide[256];
  __shared__ double shd[4];
  const int j = find_job(L.boff_t, L.n, blockIdx.x);
  const TmvJob t = L.tmv[j];
  if (t.nv <= 0) return;
  const Stage s = L.st[j];
  if (*s.status & kStFatal) return;
  const double* x1 = t.nv > 1 ? t.x[1] : t.x[0];
  const double* x2 = t.nv > 2 ? t.x[2] : t.x[0];
  const int K = s.counts[0];
  const int c = (blockIdx.x - L.boff_t[j]) * 256 + threadIdx.x;
  if (threadIdx.x == 0) nwide = 0;
  __syncthreads();
  if (c < K) {
    const int sz = s.csize[c];
    if (sz > kWideDots) {
      wide[atomicAdd(&nwide, 1)] = c;
    } else if (sz >= 2) {
      const int f = s.cfirst[c];
      double a[3];
      householder_dots_member_sum(s, f, f + sz, 0, 1, t.nv, t.x[0], x1, x2, a);
      s.hx[3 * c] = a[0];
      s.hx[3 * c + 1] = a[1];
      s.hx[3 * c + 2] = a[2];
    }
  }
  __syncthreads();
  for (int q = 0; q < nwide; ++q) {
    const int cw = wide[q], f = s.cfirst[cw];
    double a[3];
    householder_dots_member_sum(s, f, f + s.csize[cw], threadIdx.x, blockDim.x, t.nv, t.x[0], x1, x2, a);
    for (int v = 0; v < 3; ++v) {
      const double r = block_sum(a[v], shd);
      if (threadIdx.x == 0) s.hx[3 * cw + v] = r;
    }
  }
}

// Block shapes as in the secular kernel: 256 threads (boff_i) when every order
// of the level is at most kGroupMaxN, else four item blocks of one job (boff_s).
// The row poles and weights are copied into LDS first for orders up to the
// block's room; the vectors stream from global memory.
constexpr int kTmvLdsN = 8192;

template <int BT>
__global__ __launch_bounds__(BT) void cauchy_tmatvec_kernel(StageLevel L) {
  constexpr int CAP = BT == 1024 ? kTmvLdsN : kGroupMaxN;
  __shared__ double sm[2 * CAP];   // row poles, then weights
  const int* boff = BT == 1024 ? L.boff_s : L.boff_i;
  const int j = find_job(boff, L.n, blockIdx.x);
  const TmvJob t = L.tmv[j];
  if (t.nv <= 0) return;
  const Stage s = L.st[j];
  const CauchyDesc d = desc_of(s);
  const double* x1 = t.nv > 1 ? t.x[1] : t.x[0];
  const double* x2 = t.nv > 2 ? t.x[2] : t.x[0];
  const int b = (blockIdx.x - boff[j]) * (BT / 256) + (threadIdx.x >> 8), tt = threadIdx.x & 255;
  const int item = s.N <= kGroupMaxN ? b * (256 / kSmallGroup) + tt / kSmallGroup : b * 4 + (tt >> 6);
  if (s.N <= CAP) {
    for (int e = threadIdx.x; e < s.N; e += blockDim.x) {
      sm[e] = gld(d.rg + e);
      sm[CAP + e] = gld(d.rzeta + e);
    }
    __syncthreads();
    if (s.N <= kGroupMaxN)
      cauchy_tmatvec_body<kSmallGroup, true>(d, sm, sm + CAP, s.hx, t.nv, t.x[0], x1, x2, t.y[0], t.y[1], t.y[2],
                                             item);
    else
      cauchy_tmatvec_body<64, true>(d, sm, sm + CAP, s.hx, t.nv, t.x[0], x1, x2, t.y[0], t.y[1], t.y[2], item);
  } else {
    cauchy_tmatvec_body<64, false>(d, d.rg, d.rzeta, s.hx, t.nv, t.x[0], x1, x2, t.y[0], t.y[1], t.y[2], item);
  }
}

void launch_cauchy_tmatvec_level(const StageLevel& L, hipStream_t st) {
  if (L.n <= 0 || !L.tmv || L.blocks_i <= 0) return;
  hipLaunchKernelGGL(householder_dots, dim3(L.blocks_t), dim3(256), 0, st, L);
  if (L.nmax <= kGroupMaxN)
    hipLaunchKernelGGL(cauchy_tmatvec_kernel<256>, dim3(L.blocks_i), dim3(256), 0, st, L);
  else
    hipLaunchKernelGGL(cauchy_tmatvec_kernel<1024>, dim3(L.blocks_s), dim3(1024), 0, st, L);
}

}  // namespace svdu
