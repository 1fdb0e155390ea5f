// Precision form of the product X C~ (split FP32 on the matrix cores) and
// its FP64 column renormalisation sweep.
#include <stdint.h>

#include "cauchy_tile.h"
#include "jobs.h"

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

template <int MB, int NC, bool LIVE>
__device__ __forceinline__ void gemm_split32_body(const GemmJob& J, int m0, int n0, const ColDesc (&cc)[NC],
                                                  float2* Bs0, float2* Bs1) {
  constexpr int BN = 64 * NC, NB = 4 * NC;
  const CauchyDesc& d = J.d;
  const int N = d.N, R = J.R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = 4 * (lane >> 4);
  const double* xr[MB];
  bool rok[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int r = m0 + wave * 16 * MB + mb * 16 + (lane & 15);
    rok[mb] = r < R;
    xr[mb] = J.X + (size_t)(rok[mb] ? r : 0) * J.ldx;
  }
  d4 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  double aX[MB][4], bg[4][NC];
  auto loadA = [&](int k0) {
    const int kb = k0 + kq;
    if (J.vec_a && k0 + kBK <= N) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const double2 v0 = *reinterpret_cast<const double2*>(xr[mb] + kb);
        const double2 v1 = *reinterpret_cast<const double2*>(xr[mb] + kb + 2);
        aX[mb][0] = rok[mb] ? v0.x : 0.0;
        aX[mb][1] = rok[mb] ? v0.y : 0.0;
        aX[mb][2] = rok[mb] ? v1.x : 0.0;
        aX[mb][3] = rok[mb] ? v1.y : 0.0;
      }
    } else {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
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
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) bg[r][c] = gen_entry<LIVE>(d, jb + r, N, cc[c], &mind);
    if (LIVE && __any(mind < 0x1p-1000)) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + r;
        const int jj = j < N ? j : N - 1;
        RowVals rv{(j < N) ? d.rzeta[jj] : 0.0, d.rg[jj], 0.0, -2};
#pragma unroll
        for (int c = 0; c < NC; ++c) bg[r][c] = general_entry(j, rv, cc[c]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) Bn[(4 * wave + r) * BN + 64 * c + lane] = split(bg[r][c]);
  };

  const int nk = (N + kBK - 1) / kBK;
  gen_store(0, Bs0);
  loadA(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const float2* Bc = (kc & 1) ? Bs1 : Bs0;
    float2* Bn = (kc & 1) ? Bs0 : Bs1;
    float ah[MB][4], al[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float2 t = split(aX[mb][s]);
        ah[mb][s] = t.x;
        al[mb][s] = t.y;
      }
    const int kn = (kc + 1 < nk) ? (kc + 1) * kBK : kc * kBK;
    loadA(kn);
    f4 a32[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) a32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float2 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bf[nb] = Bc[(kq + s) * BN + nb * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[mb][s], bf[nb].x, a32[mb][nb], 0, 0, 0);
          a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[mb][s], bf[nb].y, a32[mb][nb], 0, 0, 0);
          a32[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[mb][s], bf[nb].x, a32[mb][nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][b][v] += (double)a32[a][b][v];
    gen_store(kn, Bn);
    __syncthreads();
  }

#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = n0 + nb * 16 + (lane & 15);
    if (col >= N) continue;
    const double sc = d.colscale ? d.colscale[col] : 1.0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wave * 16 * MB + mb * 16 + 4 * (lane >> 4) + v;
        if (row < R) J.Xo[(size_t)row * J.ldo + col] = sc * acc[mb][nb][v];
      }
    }
  }
}

template <int MB, int NC>
__device__ __forceinline__ void gemm_split32_tile(const GemmList& L, int item, float2* Bs0, float2* Bs1) {
  constexpr int BM = 64 * MB, BN = 64 * NC;
  const int j = find_job(L.boff, L.n, item);
  const GemmJob J = L.job[j];
  if (*J.d.status & kStFatal) return;
  int m0, n0;
  tile_origin(item - L.boff[j], J.tiles, J.tiles_n, BM, BN, &m0, &n0);
  const int lane = threadIdx.x & 63;
  ColDesc cc[NC];
  bool live = true;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    cc[c] = load_col_tile(J.d, n0 + 64 * c + lane);
    live = live && cc[c].type == 0;
  }
  if (__syncthreads_and(live))
    gemm_split32_body<MB, NC, true>(J, m0, n0, cc, Bs0, Bs1);
  else
    gemm_split32_body<MB, NC, false>(J, m0, n0, cc, Bs0, Bs1);
}

template <int MB, int NC>
__global__ __launch_bounds__(256, 1) void gemm_cauchy_split32_kernel(GemmList L) {
  __shared__ float2 Bs[2][kBK * 64 * NC];
  gemm_split32_tile<MB, NC>(L, blockIdx.x, Bs[0], Bs[1]);
}

template <int MB, int NC>
__global__ __launch_bounds__(256, 1) void gemm_cauchy_split32_persistent(GemmList L) {
  __shared__ float2 Bs[2][kBK * 64 * NC];
  __shared__ int next;
  if (threadIdx.x == 0) next = atomicAdd(L.counter, 1);
  __syncthreads();
  int item = next;
  while (item < L.blocks) {
    gemm_split32_tile<MB, NC>(L, item, Bs[0], Bs[1]);
    __syncthreads();
    if (threadIdx.x == 0) next = atomicAdd(L.counter, 1);
    __syncthreads();
    item = next;
  }
}

namespace {
template <int MB, int NC>
void launch_shape32(const GemmList& L, bool persistent, int grid_cap, hipStream_t st) {
  if (persistent) {
    const int g = L.blocks < grid_cap ? L.blocks : grid_cap;
    hipLaunchKernelGGL((gemm_cauchy_split32_persistent<MB, NC>), dim3(g), dim3(256), 0, st, L);
  } else {
    hipLaunchKernelGGL((gemm_cauchy_split32_kernel<MB, NC>), dim3(L.blocks), dim3(256), 0, st, L);
  }
}
}  // namespace

void launch_gemm_split32(const GemmList& L, int shape, bool persistent, int grid_cap, hipStream_t st) {
  if (L.n <= 0 || L.blocks <= 0) return;
  switch (shape) {
    case kT64x128: launch_shape32<1, 2>(L, persistent, grid_cap, st); break;
    case kT128x64: launch_shape32<2, 1>(L, persistent, grid_cap, st); break;
    case kT64x64: launch_shape32<1, 1>(L, persistent, grid_cap, st); break;
    default: launch_shape32<2, 2>(L, persistent, grid_cap, st); break;
  }
}

// ---------------------------------------------------------------------------
// FP64 refinement sweep of the precision form: every column of X (R x N) is
// rescaled to unit FP64 norm (column sums of squares in per-chunk partials,
// reduced in fixed order).
// ---------------------------------------------------------------------------
__device__ void colsumsq_body(const RenormJob& J, int cb, int chunk) {
  const int j = cb * 256 + threadIdx.x;
  const int r0 = chunk * 128, r1 = min(J.R, r0 + 128);
  if (j >= J.N) return;
  double s = 0.0;
  for (int r = r0; r < r1; ++r) {
    const double x = J.X[(size_t)r * J.ld + j];
    s += x * x;
  }
  J.part[(size_t)chunk * J.N + j] = s;
}

__device__ void colscale_body(const RenormJob& J, int cb, int chunk) {
  if (*J.status & kStFatal) return;
  const int j = cb * 256 + threadIdx.x;
  if (j >= J.N) return;
  double s = 0.0;
  for (int c = 0; c < J.chunks; ++c) s += J.part[(size_t)c * J.N + j];
  const double f = (s > 0.0) ? 1.0 / sqrt(s) : 1.0;
  const int r0 = chunk * 128, r1 = min(J.R, r0 + 128);
  for (int r = r0; r < r1; ++r) J.X[(size_t)r * J.ld + j] *= f;
}

__global__ __launch_bounds__(256) void colsumsq_partial(RenormList L) {
  const int j = find_job(L.boff, L.n, blockIdx.x);
  const RenormJob J = L.job[j];
  const int b = blockIdx.x - L.boff[j];
  colsumsq_body(J, b % J.cblocks, b / J.cblocks);
}

__global__ __launch_bounds__(256) void colscale_apply(RenormList L) {
  const int j = find_job(L.boff, L.n, blockIdx.x);
  const RenormJob J = L.job[j];
  const int b = blockIdx.x - L.boff[j];
  colscale_body(J, b % J.cblocks, b / J.cblocks);
}

size_t renorm_scratch_elems(int R, int N) { return (size_t)((R + 127) / 128) * (N > 0 ? N : 1); }

void launch_column_renorm(const RenormList& L, hipStream_t st) {
  if (L.n <= 0 || L.blocks <= 0) return;
  hipLaunchKernelGGL(colsumsq_partial, dim3(L.blocks), dim3(256), 0, st, L);
  hipLaunchKernelGGL(colscale_apply, dim3(L.blocks), dim3(256), 0, st, L);
}

namespace {
template <int MB, int NC>
int resident_blocks_gemm_split32_grid_cap() {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_cauchy_split32_persistent<MB, NC>, 256, 0) != hipSuccess) return 0;
  return nb * cus;
}
}  // namespace

// Blocks of the persistent kernel of `shape` that fit on the current device
// at once (0 if the runtime cannot tell).
int gemm_split32_grid_cap(int shape) {
  switch (shape) {
    case kT64x128: return resident_blocks_gemm_split32_grid_cap<1, 2>();
    case kT128x64: return resident_blocks_gemm_split32_grid_cap<2, 1>();
    case kT64x64: return resident_blocks_gemm_split32_grid_cap<1, 1>();
    default: return resident_blocks_gemm_split32_grid_cap<2, 2>();
  }
}

}  // namespace svdu
