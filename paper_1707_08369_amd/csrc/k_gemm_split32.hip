// Precision form of the product X C~ (split FP32 on the matrix cores) and
// its FP64 column renormalisation sweep.
#include <stdint.h>

#include "cauchy_tile.h"

namespace svdu {

// ---------------------------------------------------------------------------
// Precision form of the product: split FP32.
//
// X = Xh + Xl and C~ = Ch + Cl with Xh = fp32(X), Xl = fp32(X - Xh) (same for
// C~); X C~ ~ Xh Ch + Xh Cl + Xl Ch, three v_mfma_f32_16x16x4f32 per block
// and K sub-step. The FP32 accumulators are drained into FP64 registers after
// every K step of 16 and cleared. The tile generation, the descriptors and
// everything before the product stay FP64. Same block/wave layout as the FP64
// kernel; C~ is staged in LDS as (hi, lo) float pairs. The f32 MFMA result
// register v holds D[4 (l/16) + v][l % 16].
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool LIVE>
__device__ __forceinline__ void gemm_split32_body(int R, const double* __restrict__ X, int ldx,
                                                  const CauchyDesc& d, double* __restrict__ Xo, int ldo,
                                                  int vec_a, int m0, int n0, const ColDesc& c0,
                                                  const ColDesc& c1, float2* Bs0, float2* Bs1) {
  const int N = d.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = 4 * (lane >> 4);
  const double* xr[2];
  bool rok[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const int r = m0 + wave * 32 + mb * 16 + (lane & 15);
    rok[mb] = r < R;
    xr[mb] = X + (size_t)(rok[mb] ? r : 0) * ldx;
  }
  d4 acc[2][8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  double aX[2][4], bg[4][2];
  auto loadA = [&](int k0) {
    const int kb = k0 + kq;
    if (vec_a && k0 + kBK <= N) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const double2 v0 = *reinterpret_cast<const double2*>(xr[mb] + kb);
        const double2 v1 = *reinterpret_cast<const double2*>(xr[mb] + kb + 2);
        aX[mb][0] = rok[mb] ? v0.x : 0.0;
        aX[mb][1] = rok[mb] ? v0.y : 0.0;
        aX[mb][2] = rok[mb] ? v1.x : 0.0;
        aX[mb][3] = rok[mb] ? v1.y : 0.0;
      }
    } else {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kb + s;
          const double v = xr[mb][k < N ? k : (N - 1)];
          aX[mb][s] = (rok[mb] && k < N) ? v : 0.0;
        }
    }
  };
  auto split = [](double x) {
    const float h = (float)x;
    return float2{h, (float)(x - (double)h)};
  };
  auto gen_store = [&](int kn, float2* Bn) {
    double mind = 1.0;
    const int jb = kn + 4 * wave;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bg[r][0] = gen_entry<LIVE>(d, jb + r, N, c0, &mind);
      bg[r][1] = gen_entry<LIVE>(d, jb + r, N, c1, &mind);
    }
    if (LIVE && __any(mind < 0x1p-1000)) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + r;
        const int jj = j < N ? j : N - 1;
        RowVals rv{(j < N) ? d.rzeta[jj] : 0.0, d.rg[jj], 0.0, -2};
        bg[r][0] = general_entry(j, rv, c0);
        bg[r][1] = general_entry(j, rv, c1);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Bn[(4 * wave + r) * kBN + lane] = split(bg[r][0]);
      Bn[(4 * wave + r) * kBN + 64 + lane] = split(bg[r][1]);
    }
  };

  const int nk = (N + kBK - 1) / kBK;
  gen_store(0, Bs0);
  loadA(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const float2* Bc = (kc & 1) ? Bs1 : Bs0;
    float2* Bn = (kc & 1) ? Bs0 : Bs1;
    float ah[2][4], al[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float2 t = split(aX[mb][s]);
        ah[mb][s] = t.x;
        al[mb][s] = t.y;
      }
    const int kn = (kc + 1 < nk) ? (kc + 1) * kBK : kc * kBK;
    loadA(kn);
    f4 a32[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b) a32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float2 bf[8];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) bf[nb] = Bc[(kq + s) * kBN + nb * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[mb][s], bf[nb].x, a32[mb][nb], 0, 0, 0);
          a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[mb][s], bf[nb].y, a32[mb][nb], 0, 0, 0);
          a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[mb][s], bf[nb].x, a32[mb][nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][b][v] += (double)a32[a][b][v];
    gen_store(kn, Bn);
    __syncthreads();
  }

#pragma unroll
  for (int nb = 0; nb < 8; ++nb) {
    const int col = n0 + nb * 16 + (lane & 15);
    if (col >= N) continue;
    const double sc = d.colscale ? d.colscale[col] : 1.0;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wave * 32 + mb * 16 + 4 * (lane >> 4) + v;
        if (row < R) Xo[(size_t)row * ldo + col] = sc * acc[mb][nb][v];
      }
    }
  }
}

__global__ __launch_bounds__(256, 1) void gemm_cauchy_split32_kernel(int R, const double* __restrict__ X, int ldx,
                                                                     CauchyDesc d, double* __restrict__ Xo,
                                                                     int ldo, int vec_a) {
  __shared__ float2 Bs[2][kBK * kBN];
  if (*d.status & kStFatal) return;
  const int N = d.N;
  int m0, n0;
  tile_origin(N, &m0, &n0);
  const int lane = threadIdx.x & 63;
  const ColDesc c0 = load_col(d, n0 + lane);
  const ColDesc c1 = load_col(d, n0 + 64 + lane);
  const bool live = __syncthreads_and((c0.type == 0) && (c1.type == 0));
  if (live)
    gemm_split32_body<true>(R, X, ldx, d, Xo, ldo, vec_a, m0, n0, c0, c1, Bs[0], Bs[1]);
  else
    gemm_split32_body<false>(R, X, ldx, d, Xo, ldo, vec_a, m0, n0, c0, c1, Bs[0], Bs[1]);
}

void launch_gemm_cauchy_split32(int R, const double* X, int ldx, const CauchyDesc& d, double* Xo, int ldo,
                                hipStream_t st) {
  if (R <= 0 || d.N <= 0) return;
  const int tm = (R + kBM - 1) / kBM, tn = (d.N + kBN - 1) / kBN;
  const int vec_a = ((ldx % 2) == 0 && (reinterpret_cast<uintptr_t>(X) % 16) == 0) ? 1 : 0;
  hipLaunchKernelGGL(gemm_cauchy_split32_kernel, dim3(tm * tn), dim3(256), 0, st, R, X, ldx, d, Xo, ldo, vec_a);
}

// ---------------------------------------------------------------------------
// FP64 refinement sweep of the precision form: every column of X (R x N) is
// rescaled to unit FP64 norm (column sums of squares in per-chunk partials,
// reduced in fixed order).
// ---------------------------------------------------------------------------
__global__ void colsumsq_partial(int R, int N, const double* __restrict__ X, int ldx, double* __restrict__ part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * 128, r1 = min(R, r0 + 128);
  if (j >= N) return;
  double s = 0.0;
  for (int r = r0; r < r1; ++r) {
    const double x = X[(size_t)r * ldx + j];
    s += x * x;
  }
  part[(size_t)blockIdx.y * N + j] = s;
}

__global__ void colscale_apply(int R, int N, double* __restrict__ X, int ldx, const double* __restrict__ part,
                               int chunks, const int* status) {
  if (*status & kStFatal) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(size_t)c * N + j];
  const double f = (s > 0.0) ? 1.0 / sqrt(s) : 1.0;
  const int r0 = blockIdx.y * 128, r1 = min(R, r0 + 128);
  for (int r = r0; r < r1; ++r) X[(size_t)r * ldx + j] *= f;
}

size_t renorm_scratch_elems(int R, int N) { return (size_t)((R + 127) / 128) * (N > 0 ? N : 1); }

void launch_column_renorm(int R, int N, double* X, int ldx, double* scratch, const int* status, hipStream_t st) {
  if (R <= 0 || N <= 0) return;
  const int chunks = (R + 127) / 128;
  dim3 grid((N + 255) / 256, chunks);
  hipLaunchKernelGGL(colsumsq_partial, grid, dim3(256), 0, st, R, N, X, ldx, scratch);
  hipLaunchKernelGGL(colscale_apply, grid, dim3(256), 0, st, R, N, X, ldx, scratch, chunks, status);
}

}  // namespace svdu
