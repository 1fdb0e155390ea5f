// Projections X^T v (Algorithm Step 1 and RankOneUpdate Step 1).
//
// X is row-major R x N. One pass over X serves up to three vectors. Threads
// own columns (coalesced 2 KiB rows per block) and a block owns a chunk of
// rows; per-chunk partial sums are reduced in a second, fixed-order pass so
// that results are bitwise reproducible. HBM-bound: 8 R N bytes per pass.
#include "device_util.h"
#include "jobs.h"
#include "svdu_internal.h"

namespace svdu {

constexpr int kGemvCols = 256;
constexpr int kGemvRows = 128;

__device__ void gemv_t_partial_body(int R, int N, const double* __restrict__ X, int ldx, int nv,
                                    const double* __restrict__ v0, const double* __restrict__ v1,
                                    const double* __restrict__ v2, double* __restrict__ part, int cb, int chunk) {
  const int j = cb * kGemvCols + threadIdx.x;
  const int r0 = chunk * kGemvRows;
  const int r1 = min(R, r0 + kGemvRows);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (j < N) {
    const double* xp = X + (size_t)r0 * ldx + j;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
      const double x0 = xp[0], x1 = xp[(size_t)ldx], x2 = xp[2 * (size_t)ldx], x3 = xp[3 * (size_t)ldx];
      a0 += x0 * v0[r];
      a0 += x1 * v0[r + 1];
      a0 += x2 * v0[r + 2];
      a0 += x3 * v0[r + 3];
      if (nv > 1) {
        a1 += x0 * v1[r];
        a1 += x1 * v1[r + 1];
        a1 += x2 * v1[r + 2];
        a1 += x3 * v1[r + 3];
      }
      if (nv > 2) {
        a2 += x0 * v2[r];
        a2 += x1 * v2[r + 1];
        a2 += x2 * v2[r + 2];
        a2 += x3 * v2[r + 3];
      }
      xp += 4 * (size_t)ldx;
    }
    for (; r < r1; ++r) {
      const double x = *xp;
      a0 += x * v0[r];
      if (nv > 1) a1 += x * v1[r];
      if (nv > 2) a2 += x * v2[r];
      xp += ldx;
    }
    double* p = part + (size_t)chunk * nv * N;
    p[j] = a0;
    if (nv > 1) p[N + j] = a1;
    if (nv > 2) p[2 * (size_t)N + j] = a2;
  }
}

__device__ void gemv_t_reduce_body(int N, int nv, int chunks, const double* __restrict__ part, double* out0,
                                   double* out1, double* out2, int idx) {
  if (idx >= nv * N) return;
  const int k = idx / N, j = idx - k * N;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[((size_t)c * nv + k) * N + j];
  double* o = (k == 0) ? out0 : (k == 1) ? out1 : out2;
  o[j] = s;
}

__global__ __launch_bounds__(kGemvCols) void gemv_t_partial(GemvList L) {
  const int j = find_job(L.boff_p, L.n, blockIdx.x);
  const GemvJob J = L.job[j];
  const int b = blockIdx.x - L.boff_p[j];
  const double* v1 = J.nv > 1 ? J.v[1] : J.v[0];
  const double* v2 = J.nv > 2 ? J.v[2] : J.v[0];
  gemv_t_partial_body(J.R, J.N, J.X, J.ldx, J.nv, J.v[0], v1, v2, J.part, b % J.cblocks, b / J.cblocks);
}

__global__ __launch_bounds__(256) void gemv_t_reduce(GemvList L) {
  const int j = find_job(L.boff_r, L.n, blockIdx.x);
  const GemvJob J = L.job[j];
  gemv_t_reduce_body(J.N, J.nv, J.chunks, J.part, J.out[0], J.out[1], J.out[2],
                     (blockIdx.x - L.boff_r[j]) * 256 + threadIdx.x);
}

int gemv_cblocks(int N) { return (N + kGemvCols - 1) / kGemvCols; }
int gemv_chunks(int R) { return (R + kGemvRows - 1) / kGemvRows; }

size_t gemv_t_scratch_elems(int R, int N, int nv) {
  const int chunks = (R + kGemvRows - 1) / kGemvRows;
  return (size_t)(chunks > 0 ? chunks : 1) * nv * N;
}

void launch_gemv_list(const GemvList& L, hipStream_t st) {
  if (L.n <= 0 || L.blocks_p <= 0) return;
  hipLaunchKernelGGL(gemv_t_partial, dim3(L.blocks_p), dim3(kGemvCols), 0, st, L);
  hipLaunchKernelGGL(gemv_t_reduce, dim3(L.blocks_r), dim3(256), 0, st, L);
}

}  // namespace svdu
