// Products with the Cauchy eigenvector matrix C~ of one eigen-update:
// y = C~^T x for up to three vectors. It carries the projected vectors between
// the two eigen-updates of one side in core space (z for the second update is
// C~^T of the first applied to U^T b1, since U~^T b1 = C~^T U^T b1) and maps
// the sign probes.
#include "cauchy_tile.h"

namespace svdu {

// ---------------------------------------------------------------------------
// y = C~^T x
// ---------------------------------------------------------------------------
__global__ void householder_dots(Stage s, int nv, const double* x0, const double* x1, const double* x2) {
  if (*s.status & kStFatal) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = s.counts[0];
  if (c >= K) return;
  const int sz = s.csize[c];
  if (sz < 2) return;
  const int f = s.cfirst[c];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = f; k < f + sz; ++k) {
    const int j = s.col_of[s.Llist[k]];
    const double h = s.rh[j];
    a0 += h * x0[j];
    if (nv > 1) a1 += h * x1[j];
    if (nv > 2) a2 += h * x2[j];
  }
  s.hx[3 * c] = a0;
  s.hx[3 * c + 1] = a1;
  s.hx[3 * c + 2] = a2;
}

__global__ __launch_bounds__(256) void cauchy_tmatvec_kernel(CauchyDesc d, const double* __restrict__ hx, int nv,
                                                             const double* __restrict__ x0,
                                                             const double* __restrict__ x1,
                                                             const double* __restrict__ x2, double* y0,
                                                             double* y1, double* y2) {
  if (*d.status & kStFatal) return;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= d.N) return;
  const ColDesc cd = load_col(d, c);
  if (cd.type == 0) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int j = lane; j < d.N; j += 64) {
      const double z = d.rzeta[j];
      if (z == 0.0) continue;
      const double w = z * recip((d.rg[j] - cd.o) - cd.t);
      a0 += w * x0[j];
      if (nv > 1) a1 += w * x1[j];
      if (nv > 2) a2 += w * x2[j];
    }
    a0 = wave_sum(a0);
    if (nv > 1) a1 = wave_sum(a1);
    if (nv > 2) a2 = wave_sum(a2);
    if (lane == 0) {
      y0[c] = cd.s * a0;
      if (nv > 1) y1[c] = cd.s * a1;
      if (nv > 2) y2[c] = cd.s * a2;
    }
  } else if (lane == 0 && cd.mem >= 0 && cd.mem < d.N) {
    const bool hh = cd.h != 0.0 && cd.cl >= 0 && cd.cl < d.N;
    y0[c] = x0[cd.mem] - (hh ? 2.0 * cd.h * hx[3 * cd.cl] : 0.0);
    if (nv > 1) y1[c] = x1[cd.mem] - (hh ? 2.0 * cd.h * hx[3 * cd.cl + 1] : 0.0);
    if (nv > 2) y2[c] = x2[cd.mem] - (hh ? 2.0 * cd.h * hx[3 * cd.cl + 2] : 0.0);
  }
}

void launch_cauchy_tmatvec(const Stage& s, int nv, const double* const* x, double* const* y, hipStream_t st) {
  const int N = s.N;
  if (N <= 0) return;
  const double* x1 = nv > 1 ? x[1] : x[0];
  const double* x2 = nv > 2 ? x[2] : x[0];
  double* y1 = nv > 1 ? y[1] : nullptr;
  double* y2 = nv > 2 ? y[2] : nullptr;
  hipLaunchKernelGGL(householder_dots, dim3((N + 255) / 256), dim3(256), 0, st, s, nv, x[0], x1, x2);
  hipLaunchKernelGGL(cauchy_tmatvec_kernel, dim3((N + 3) / 4), dim3(256), 0, st, desc_of(s), s.hx, nv, x[0], x1,
                     x2, y[0], y1, y2);
}

}  // namespace svdu
