// Deflated output columns of a product X C~ without the MFMA loop, shared by
// the FP64 and the exact-slice INT8 product kernels.
//
// A deflated column c of C~ is a unit vector e_mem, or one column of the
// Householder reflection of its cluster (RankOneUpdate, deflation of repeated
// poles):
//   X C~[:, c] = X[:, mem] - 2 h_c sum_{j in cluster} rh_j X[:, j].
// A 64-column chunk (aligned to 64 in the output) takes this path when every
// in-range column of it is deflated and all its reflected columns belong to
// one cluster. The test depends only on the chunk's descriptors, and the row
// sums below have a fixed order, so a column's value does not depend on the
// tile shape, the schedule, the batch or the product kernel. Every wave holds
// the same 64 columns, so the test is a wave-level reduction with a
// block-uniform result.
//
// The job type Job has R, X, ldx, Xo, ldo and d (CauchyDesc with members).
#pragma once
#include "cauchy_tile.h"

namespace svdu {

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Mask of the chunks that take the copy path; cl[c] is the chunk's cluster
// (-1: unit columns only).
template <int NC>
__device__ __forceinline__ unsigned copy_chunks(const CauchyDesc& d, int n0, const ColDesc (&cc)[NC], int (&cl)[NC]) {
  if (d.Llist == nullptr) return 0u;
  const int lane = threadIdx.x & 63;
  const int K = gld(d.counts);
  unsigned mask = 0u;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const bool in = n0 + 64 * c + lane < d.N;
    const bool refl = in && cc[c].type == 1 && cc[c].h != 0.0 && cc[c].cl >= 0;
    const bool bad = in && (cc[c].type != 1 || cc[c].mem < 0 || cc[c].mem >= d.N || (refl && cc[c].cl >= K));
    const int key = refl ? cc[c].cl : -1;
    const int kmax = wave_max_int(key);
    cl[c] = kmax;
    if (n0 + 64 * c < d.N && !group_any<64>(bad || (refl && key != kmax))) mask |= 1u << c;
  }
  return mask;
}

// dots[rr] = sum over the members j of cluster cl of rh_j X[m0 + rr, j], for
// the BM rows of the tile (T threads). Eight lanes share a row; lane t takes
// the members q = t (mod 8) in increasing order, then the eight partial sums
// are added by a butterfly. Members are staged through LDS in chunks of S.
template <int BM, int T, int S, class Job>
__device__ __forceinline__ void cluster_dots(const Job& J, int m0, int cl, double* rhs, int* js, double* dots) {
  constexpr int RPP = T / 8, NP = BM / RPP;
  static_assert(BM % RPP == 0, "row passes");
  const CauchyDesc& d = J.d;
  const int tid = threadIdx.x, t8 = tid & 7;
  const int f = gld(d.cfirst + cl);
  int sz = gld(d.csize + cl);
  if (f < 0 || sz < 0 || f + sz > d.N) sz = 0;   // never from a valid stage; keeps every index in range
  double acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.0;
  for (int q0 = 0; q0 < sz; q0 += S) {
    const int len = min(S, sz - q0);
    __syncthreads();   // LDS free: the product's buffers, or the previous member chunk
    for (int q = tid; q < len; q += T) {
      const int t = min(max(gld(d.Llist + f + q0 + q), 0), d.N - 1);
      const int j = min(max(gld(d.col_of + t), 0), d.N - 1);
      js[q] = j;
      rhs[q] = gld(d.rh + j);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int r = m0 + p * RPP + (tid >> 3);
      if (r < J.R) {
        const double* xr = J.X + (size_t)r * J.ldx;
        double a = acc[p];
#pragma unroll 4
        for (int q = t8; q < len; q += 8) a = __builtin_fma(rhs[q], gld(xr + js[q]), a);
        acc[p] = a;
      }
    }
  }
  __syncthreads();   // the last member chunk has been read
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const double a = group_sum<8>(acc[p]);
    if (t8 == 0) dots[p * RPP + (tid >> 3)] = a;
  }
  __syncthreads();
}

// The chunks of `mask` of a BM x 64 NC tile (T threads, W = T / 64 waves):
// rhs and js hold S members, dots BM row sums (LDS).
template <int BM, int T, int NC, int S, class Job>
__device__ __forceinline__ void copy_path(const Job& J, int m0, int n0, const ColDesc (&cc)[NC],
                                          const int (&cl)[NC], unsigned mask, double* rhs, int* js,
                                          double* dots) {
  constexpr int W = T / 64;
  const CauchyDesc& d = J.d;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int have = -1;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!((mask >> c) & 1u)) continue;
    if (cl[c] >= 0 && cl[c] != have) {
      cluster_dots<BM, T, S>(J, m0, cl[c], rhs, js, dots);
      have = cl[c];
    }
    const int col = n0 + 64 * c + lane;
    if (col >= d.N) continue;
    const double sc = d.colscale ? gld(d.colscale + col) : 1.0;
    const bool refl = cc[c].h != 0.0 && cc[c].cl >= 0;
    const double h2 = -2.0 * cc[c].h;
    for (int rr = wave; rr < BM; rr += W) {
      const int r = m0 + rr;
      if (r >= J.R) break;
      const double x = gld(J.X + (size_t)r * J.ldx + cc[c].mem);
      const double v = refl ? __builtin_fma(h2, dots[rr], x) : x;
      gst(J.Xo + (size_t)r * J.ldo + col, sc * v);
    }
  }
}

}  // namespace svdu
