// X_out = X C~ in FP64 on the matrix cores (RankOneUpdate Steps 4-7,
// equation UCTildeProduct): the dense product of the direct path, with the
// C~ tiles regenerated from O(N) descriptors and never stored in HBM.
//
// One launch serves a list of products (GemmList). W waves (4 or 8) are
// stacked along M: wave w owns 16 MB rows of the block tile and all of its
// 64 NC columns, so no wave loads the X rows of another. K advances 16 per
// half-step.
// X fragments come straight from HBM into registers one step ahead, in a
// K-permuted layout: in MFMA step s, lane l supplies X[row][k0 + 4 (l/16) + s]
// (four consecutive doubles of one row per lane) and the matching entry
// C~[k0 + 4 (l/16) + s][col]; the contraction covers all 16 k either way.
// Two register sets are used alternately (the K loop is unrolled by two). C~
// tiles are double-buffered in LDS in stages of KH half-steps, one barrier
// per stage. Each wave generates 16 / W rows of every half-step KH ahead,
// interleaved with its MFMAs. The generation is VALU work that the matrix
// core does not hide, so its share of the time falls with the rows of X each
// generated entry serves: 8 waves (256 rows) halve it against 4 waves.
// A block whose columns are all secular roots (the usual case) runs the
// Cauchy formula without any branch; other blocks use the general entry,
// which gives the same values. Out-of-range rows of X load row 0 instead of
// zeros: their accumulators are never stored. Chunks of 64 deflated columns
// (the zero block of a rectangular problem, for one) are written as copies
// and one reflection instead; a block made only of such chunks runs no MFMA.
//
// Every output element is accumulated by the same sequence of MFMAs (the
// K order and permutation do not depend on the tile shape or on the other
// jobs), or by the same copy-path sum, so the result is bitwise the same for
// every tile shape, schedule and batch composition.
//
// MFMA v_mfma_f64_16x16x4f64 operand layout (lane l): A[l % 16][l / 16],
// B[l / 16][l % 16]; result register v holds D[l / 16 + 4 v][l % 16].
#include <stdint.h>

#include <type_traits>

#include "cauchy_tile.h"
#include "copy_path.h"
#include "jobs.h"

namespace svdu {

// Live entry of the product kernels: the refined reciprocal of live_entry,
// without its select for z = 0. A row with z = 0 either gives a signed zero
// (0 times a finite reciprocal) or has |delta| below the tiny-delta bound,
// which sends the whole row group through general_entry.
__device__ __forceinline__ double prod_live_entry(double z, double g, const ColDesc& c, double* mind) {
  const double del = (g - c.o) - c.t;
  *mind = __builtin_fmin(*mind, __builtin_fabs(del));
  double r = __builtin_amdgcn_rcp(del);
  double e = __builtin_fma(-del, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-del, r, 1.0);
  r = __builtin_fma(r, e, r);
  return (z * c.s) * r;
}

template <bool LIVE>
__device__ __forceinline__ double prod_entry(const CauchyDesc& d, int j, int N, const ColDesc& c, double* mind) {
  if (!LIVE) return gen_entry<false>(d, j, N, c, mind);
  const int jj = j < N ? j : N - 1;
  const double zl = gld(d.rzeta + jj);
  const double z = (j < N) ? zl : 0.0;
  return prod_live_entry(z, gld(d.rg + jj), c, mind);
}

// `skip`: 64-column chunks of the tile whose results are not stored (the
// copy path below writes them); always 0 for an all-live block.
template <int MB, int NC, int KH, int W, bool LIVE>
__device__ __forceinline__ void gemm_f64_body(const GemmJob& J, int m0, int n0, const ColDesc (&cc)[NC],
                                              double* Bs0, double* Bs1, unsigned skip) {
  // RPW: C~ rows each wave generates per half-step; SPR: MFMA groups per row
  constexpr int BN = 64 * NC, NB = 4 * NC, RPW = 16 / W, SPR = 4 / RPW;
  static_assert(W == 4 || W == 8, "4 or 8 waves");
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
    xr[mb] = J.X + (size_t)(rok[mb] ? r : 0) * J.ldx;   // rows past R read row 0; never stored
  }
  d4 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  double aA[MB][4], aB[MB][4], bg[RPW][NC];
  // X of the half-step at k index k0: 16-byte loads (aligned rows, the whole
  // step in range), or element loads with the tail zeroed
  auto loadA_vec = [&](int k0, double (&a)[MB][4]) {
    const int kb = k0 + kq;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const double2 v0 = gld2(xr[mb] + kb);
      const double2 v1 = gld2(xr[mb] + kb + 2);
      a[mb][0] = v0.x;
      a[mb][1] = v0.y;
      a[mb][2] = v1.x;
      a[mb][3] = v1.y;
    }
  };
  auto loadA = [&](int k0, double (&a)[MB][4]) {
    const int kb = k0 + kq;
    if (J.vec_a && k0 + kBK <= N) {   // block-uniform: the whole step is in range
      loadA_vec(k0, a);
    } else {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kb + s;
          const double v = gld(xr[mb] + (k < N ? k : (N - 1)));
          a[mb][s] = (rok[mb] && k < N) ? v : 0.0;
        }
    }
  };
  // entries of C~ rows jb .. jb + RPW - 1 for this lane's NC columns
  auto fix_tiny = [&](int jb) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = jb + r;
      const int jj = j < N ? j : N - 1;
      RowVals rv{(j < N) ? gld(d.rzeta + jj) : 0.0, gld(d.rg + jj), 0.0, -2};
#pragma unroll
      for (int c = 0; c < NC; ++c) bg[r][c] = general_entry(j, rv, cc[c]);
    }
  };
  auto store_b = [&](double* Bn) {
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) Bn[(RPW * wave + r) * BN + 64 * c + lane] = bg[r][c];
  };
  // Half-step hs covers k in [16 hs, 16 hs + 16). The LDS buffers hold KH
  // half-steps each; half-step hs is row block hs % KH of buffer (hs / KH) % 2.
  auto bufof = [&](int hs) { return (((hs / KH) & 1) ? Bs1 : Bs0) + (hs % KH) * kBK * BN; };
  // Row descriptors (zeta, g) of the C~ rows a wave generates in half-step
  // hs (rows (hs + KH) kBK + RPW wave + r). On the all-live path of the
  // 8-wave tile (PRE) they are loaded one half-step ahead, before that step's
  // X: loads complete in the order issued as far as the wait counter is
  // concerned, so a wait for the descriptors of this half-step never waits
  // for the X of the next one, and X has a whole half-step to arrive. The
  // 4-wave tiles have no registers to spare for them and load them where
  // they are used.
  constexpr bool PRE = LIVE && W == 8;
  auto load_desc = [&](int hs, double (&z)[RPW], double (&g)[RPW]) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = (hs + KH) * kBK + RPW * wave + r, jj = j < N ? j : N - 1;
      const double zl = gld(d.rzeta + jj);
      z[r] = (j < N) ? zl : 0.0;
      g[r] = gld(d.rg + jj);
    }
  };
  // one half-step: MFMAs on (a, C~ of hs) interleaved with generating
  // half-step hs + KH; one barrier per KH half-steps. Issues the descriptor
  // loads of half-step hs + 1 (into zn, gn) and then X of the half-step at
  // k index kpre (into an, if kpre >= 0). With VEC (std::true_type; the
  // 8-wave tile) the X load is a full 16-byte step with no branch, so the
  // wait counts the compiler places follow the issue order above.
  auto step = [&](auto VEC, const double (&a)[MB][4], int hs, double (&an)[MB][4], int kpre,
                  const double (&zc)[RPW], const double (&gc)[RPW], double (&zn)[RPW], double (&gn)[RPW]) {
    const double* Bcur = bufof(hs);
    double* Bnext = bufof(hs + KH);
    const int kn = (hs + KH) * kBK;
    double mind = 1.0;
    const int jb = kn + RPW * wave;
    if (PRE) load_desc(hs + 1, zn, gn);
    if constexpr (decltype(VEC)::value)
      loadA_vec(kpre, an);
    else if (kpre >= 0)
      loadA(kpre, an);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bf[nb] = Bcur[(kq + s) * BN + nb * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][s], bf[nb], acc[mb][nb], 0, 0, 0);
      if (s % SPR == SPR - 1) {
        const int r = s / SPR;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          bg[r][c] = PRE ? prod_live_entry(zc[r], gc[r], cc[c], &mind) : prod_entry<LIVE>(d, jb + r, N, cc[c], &mind);
      }
    }
    if (LIVE && __any(mind < 0x1p-1000)) fix_tiny(jb);
    store_b(Bnext);
    if (hs % KH == KH - 1) __syncthreads();
  };

  const int nk = (N + kBK - 1) / kBK;
  // prologue: C~ of half-steps 0 .. KH-1 into buffer 0, X of half-step 0 into aA
#pragma unroll
  for (int h = 0; h < KH; ++h) {
    double mind = 1.0;
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) bg[r][c] = prod_entry<LIVE>(d, h * kBK + RPW * wave + r, N, cc[c], &mind);
    if (LIVE && __any(mind < 0x1p-1000)) fix_tiny(h * kBK + RPW * wave);
    store_b(bufof(h));
  }
  double zA[RPW], gA[RPW], zB[RPW], gB[RPW];
  if (PRE) load_desc(0, zA, gA);
  loadA(0, aA);
  __syncthreads();
  int kc = 0;
  if constexpr (W == 8) {
    if (J.vec_a) {
      // pairs of half-steps whose X loads (half-steps kc + 1, kc + 2) are full 16-k steps
      const int nv = N / kBK;
      for (; kc + 3 <= nv; kc += 2) {
        step(std::true_type{}, aA, kc, aB, (kc + 1) * kBK, zA, gA, zB, gB);
        step(std::true_type{}, aB, kc + 1, aA, (kc + 2) * kBK, zB, gB, zA, gA);
      }
    }
    for (; kc + 2 <= nk; kc += 2) {
      step(std::false_type{}, aA, kc, aB, (kc + 1) * kBK, zA, gA, zB, gB);
      const int k2 = (kc + 2 < nk) ? (kc + 2) * kBK : (kc + 1) * kBK;
      step(std::false_type{}, aB, kc + 1, aA, k2, zB, gB, zA, gA);
    }
  } else {
    // 4-wave tiles: X of the next half-step is loaded ahead of each step
    for (; kc + 2 <= nk; kc += 2) {
      loadA((kc + 1) * kBK, aB);
      step(std::false_type{}, aA, kc, aB, -1, zA, gA, zB, gB);
      const int k2 = (kc + 2 < nk) ? (kc + 2) * kBK : (kc + 1) * kBK;
      loadA(k2, aA);
      step(std::false_type{}, aB, kc + 1, aA, -1, zB, gB, zA, gA);
    }
  }
  if (kc < nk) step(std::false_type{}, aA, kc, aB, -1, zA, gA, zB, gB);

#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = n0 + nb * 16 + (lane & 15);
    if (col >= N || (!LIVE && ((skip >> (nb >> 2)) & 1u))) continue;
    const double sc = d.colscale ? gld(d.colscale + col) : 1.0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wave * 16 * MB + mb * 16 + (lane >> 4) + 4 * v;
        if (row < R) gst(J.Xo + (size_t)row * J.ldo + col, sc * acc[mb][nb][v]);
      }
    }
  }
}

// Deflated columns without the MFMA loop: copy_path.h.
template <int MB, int NC, int KH, int W>
__device__ __forceinline__ void copy_path(const GemmJob& J, int m0, int n0, const ColDesc (&cc)[NC],
                                          const int (&cl)[NC], unsigned mask, double* Bs0, double* Bs1) {
  constexpr int BM = 16 * MB * W, T = 64 * W, S = KH * kBK * 64 * NC;
  static_assert(2 * BM <= S, "dots and member rows share one C~ buffer");
  copy_path<BM, T, NC, S>(J, m0, n0, cc, cl, mask, Bs0, reinterpret_cast<int*>(Bs1 + BM), Bs1);
}

// One tile (work item) of a GemmList. COPY: the copy path is compiled in (for
// lists with a job that carries cluster members). The kernels without it keep
// the register allocation of the plain product; with it, the chunk test runs
// ahead of the MFMA branch, where it leaves the all-live loop's waits as in
// the plain kernels (placed after the branch, it added two vmcnt waits).
template <int MB, int NC, int KH, int W, bool COPY>
__device__ __forceinline__ void gemm_f64_tile(const GemmList& L, int item, double* Bs0, double* Bs1) {
  constexpr int BM = 16 * MB * W, BN = 64 * NC;
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
  int cl[NC];
  unsigned cp = 0u;
  if (COPY) {
    cp = copy_chunks<NC>(J.d, n0, cc, cl);
    unsigned inr = 0u;
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (n0 + 64 * c < J.d.N) inr |= 1u << c;
    if (cp && (cp & inr) == inr) {
      copy_path<MB, NC, KH, W>(J, m0, n0, cc, cl, cp, Bs0, Bs1);
      return;
    }
  }
  if (__syncthreads_and(live))
    gemm_f64_body<MB, NC, KH, W, true>(J, m0, n0, cc, Bs0, Bs1, 0u);
  else
    gemm_f64_body<MB, NC, KH, W, false>(J, m0, n0, cc, Bs0, Bs1, cp);
  if (COPY && cp) copy_path<MB, NC, KH, W>(J, m0, n0, cc, cl, cp, Bs0, Bs1);
}

// Grid schedule: one block per tile, in list order. KH half-steps of 16 k
// share one barrier (LDS buffers of 16 KH rows). Two blocks of 4 waves or one
// of 8 waves per CU: 2 waves per SIMD, 256 VGPRs each.
template <int MB, int NC, int KH, int W>
__global__ __launch_bounds__(64 * W, 8 / W) void gemm_cauchy_f64_kernel(GemmList L) {
  __shared__ double Bs[2][KH * kBK * 64 * NC];
  gemm_f64_tile<MB, NC, KH, W, false>(L, blockIdx.x, Bs[0], Bs[1]);
}
template <int MB, int NC, int KH, int W>
__global__ __launch_bounds__(64 * W, 8 / W) void gemm_cauchy_f64_copy_kernel(GemmList L) {
  __shared__ double Bs[2][KH * kBK * 64 * NC];
  gemm_f64_tile<MB, NC, KH, W, true>(L, blockIdx.x, Bs[0], Bs[1]);
}

// Persistent schedule: as many blocks as fit on the device at once; each
// takes tiles in list order from a counter until the list is exhausted.
template <int MB, int NC, int KH, int W, bool COPY>
__device__ __forceinline__ void gemm_f64_persistent_loop(const GemmList& L) {
  __shared__ double Bs[2][KH * kBK * 64 * NC];
  __shared__ int next;
  if (threadIdx.x == 0) next = atomicAdd(L.counter, 1);
  __syncthreads();
  int item = next;
  while (item < L.blocks) {
    gemm_f64_tile<MB, NC, KH, W, COPY>(L, item, Bs[0], Bs[1]);
    __syncthreads();   // every thread has read `next` and finished with Bs
    if (threadIdx.x == 0) next = atomicAdd(L.counter, 1);
    __syncthreads();
    item = next;
  }
}
template <int MB, int NC, int KH, int W>
__global__ __launch_bounds__(64 * W, 8 / W) void gemm_cauchy_f64_persistent(GemmList L) {
  gemm_f64_persistent_loop<MB, NC, KH, W, false>(L);
}
template <int MB, int NC, int KH, int W>
__global__ __launch_bounds__(64 * W, 8 / W) void gemm_cauchy_f64_copy_persistent(GemmList L) {
  gemm_f64_persistent_loop<MB, NC, KH, W, true>(L);
}

namespace {
template <int MB, int NC, int KH, int W>
void launch_shape(const GemmList& L, bool persistent, int grid_cap, hipStream_t st) {
  if (persistent) {
    const int g = L.blocks < grid_cap ? L.blocks : grid_cap;
    if (L.copy)
      hipLaunchKernelGGL((gemm_cauchy_f64_copy_persistent<MB, NC, KH, W>), dim3(g), dim3(64 * W), 0, st, L);
    else
      hipLaunchKernelGGL((gemm_cauchy_f64_persistent<MB, NC, KH, W>), dim3(g), dim3(64 * W), 0, st, L);
  } else if (L.copy) {
    hipLaunchKernelGGL((gemm_cauchy_f64_copy_kernel<MB, NC, KH, W>), dim3(L.blocks), dim3(64 * W), 0, st, L);
  } else {
    hipLaunchKernelGGL((gemm_cauchy_f64_kernel<MB, NC, KH, W>), dim3(L.blocks), dim3(64 * W), 0, st, L);
  }
}
}  // namespace

void launch_gemm_f64(const GemmList& L, int shape, bool persistent, int grid_cap, hipStream_t st) {
  if (L.n <= 0 || L.blocks <= 0) return;
  switch (shape) {
    case kT64x128: launch_shape<1, 2, 1, 4>(L, persistent, grid_cap, st); break;
    case kT128x64: launch_shape<2, 1, 1, 4>(L, persistent, grid_cap, st); break;
    case kT64x64: launch_shape<1, 1, 1, 4>(L, persistent, grid_cap, st); break;
    case kT128x128k32: launch_shape<2, 2, 2, 4>(L, persistent, grid_cap, st); break;
    case kT256x128k64: launch_shape<2, 2, 4, 8>(L, persistent, grid_cap, st); break;
    default: launch_shape<2, 2, 1, 4>(L, persistent, grid_cap, st); break;
  }
}

namespace {
template <int MB, int NC, int KH, int W>
int resident_blocks_gemm_f64_grid_cap() {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_cauchy_f64_persistent<MB, NC, KH, W>, 64 * W, 0) !=
      hipSuccess)
    return 0;
  return nb * cus;
}
}  // namespace

// Blocks of the persistent kernel of `shape` that fit on the current device
// at once (0 if the runtime cannot tell).
int gemm_f64_grid_cap(int shape) {
  switch (shape) {
    case kT64x128: return resident_blocks_gemm_f64_grid_cap<1, 2, 1, 4>();
    case kT128x64: return resident_blocks_gemm_f64_grid_cap<2, 1, 1, 4>();
    case kT64x64: return resident_blocks_gemm_f64_grid_cap<1, 1, 1, 4>();
    case kT128x128k32: return resident_blocks_gemm_f64_grid_cap<2, 2, 2, 4>();
    case kT256x128k64: return resident_blocks_gemm_f64_grid_cap<2, 2, 4, 8>();
    default: return resident_blocks_gemm_f64_grid_cap<2, 2, 1, 4>();
  }
}

}  // namespace svdu
