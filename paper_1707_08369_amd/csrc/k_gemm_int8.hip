// Precision form of the product X C~ with FP64-level accuracy on the INT8
// matrix cores (RankOneUpdate Steps 4-7, equation UCTildeProduct): exact
// slices, an Ozaki-style split.
//
// Every row of X and every column of C~ is scaled by a power of two 2^E so
// that its largest entry lies in [1/2, 1), then cut into S signed slices of
// seven bits: t_1 = 64 x 2^-E, a_s = rint(t_s), t_(s+1) = 128 (t_s - a_s).
// Every step is exact in FP64, every a_s lies in [-64, 64], and
//   x = 2^E sum_s a_s 2^(1 - 7 s)   up to |x - ...| <= 2^(E - 7 S).
// The product of a row of X and a column of C~ is then
//   sum_(s,t) 2^(Ex + Ec + 2 - 7 (s + t)) (a_s . b_t),
// where every slice dot product a_s . b_t is a sum of N products of integers
// of at most 64 in magnitude: exact in INT32 for N < 2^31 / (S 64^2) (more
// than 65000 for S = 8). The pairs with s + t <= S + 1 are kept (the dropped
// ones are below the slicing error); pairs with the same s + t share one
// INT32 accumulator, so S accumulators per output element carry every pair,
// and the epilogue combines them in FP64 (Horner in 2^-7, then one exact
// power-of-two scale).
//
// The slices of X and C~ are written once per product into HBM as 1 KiB
// tiles in the operand order of v_mfma_i32_16x16x64_i8 (jobs.h), so the
// product kernel reads each operand fragment with one 16-byte load per lane.
// Entries of C~ come from the same descriptors and the same formula as in the
// FP64 kernels, so the sliced matrix is the FP64 C~ up to the slicing error.
//
// Product kernel: 4 waves, block tile 128 x 64; wave w owns rows
// [32 w, 32 w + 32) of the tile (two MFMA row blocks) and all 64 columns
// (four column blocks), so its A fragments are its own and come straight from
// HBM into registers one k step ahead; the B fragments (4 column blocks x S
// slices per k step of 64) are shared through LDS, double-buffered, one
// barrier per step (a buffer written at step kb was last read at step kb - 2,
// before the barrier of step kb - 1). Per k step a wave issues 8 S (S + 1) / 2 MFMAs on 8 S
// accumulator registers sets of 4 (S = 7: 224 MFMAs, 224 accumulator VGPRs).
// Every output element is computed by the same sequence of operations
// whatever the batch or the launch, so results are deterministic.
//
// MFMA v_mfma_i32_16x16x64_i8 (lane l): A row l % 16, B column l % 16, each
// 16 bytes that hold k = 16 (l / 16) + 0..15 in both operands; result register
// v holds D[4 (l / 16) + v][l % 16].
#include <stdint.h>

#include "cauchy_tile.h"
#include "copy_path.h"
#include "jobs.h"

namespace svdu {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

// E with m < 2^E <= 2 m (0 for m == 0): the scale of a row or column whose
// largest magnitude is m.
__device__ __forceinline__ int scale_exp(double m) {
  if (!(m > 0.0)) return 0;
  return __builtin_amdgcn_frexp_exp(m);   // m = f 2^E, f in [1/2, 1)
}

// S slices of 16 values already scaled into (-1, 1); byte j of each 16-byte
// slice is value j.
template <int S>
__device__ __forceinline__ void slice16(const double (&x)[16], v4i (&out)[S]) {
  double t[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) t[j] = x[j] * 64.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double a = __builtin_rint(t[j]);
      t[j] = (t[j] - a) * 128.0;
      w[j >> 2] |= ((unsigned)(int)a & 0xffu) << (8 * (j & 3));
    }
    out[s] = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
  }
}

// ---------------------------------------------------------------------------
// slices of the rows of X: one block of 256 threads per 16 rows
// ---------------------------------------------------------------------------
template <int S>
__device__ void slice_x_body(const SliceXJob& J, int rb) {
  __shared__ int sexp[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = J.R, N = J.N;
  // 16-byte loads where the rows allow them (16-byte aligned rows of even length)
  const bool vec = ((reinterpret_cast<uintptr_t>(J.X) & 15) == 0) && (J.ldx % 2 == 0) && (N % 2 == 0);
  {
    // row maxima: 16 threads per row, each 16 bytes of 256 contiguous bytes per
    // step, four independent running maxima
    const int rr = tid >> 4, c0 = tid & 15, r = rb * 16 + rr;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (r < R) {
      const double* xr = J.X + (size_t)r * J.ldx;
      if (vec) {
        int c = 2 * c0;
        for (; c + 96 < N; c += 128) {
          const double2 v0 = gld2(xr + c), v1 = gld2(xr + c + 32), v2 = gld2(xr + c + 64), v3 = gld2(xr + c + 96);
          m0 = __builtin_fmax(m0, __builtin_fmax(__builtin_fabs(v0.x), __builtin_fabs(v0.y)));
          m1 = __builtin_fmax(m1, __builtin_fmax(__builtin_fabs(v1.x), __builtin_fabs(v1.y)));
          m2 = __builtin_fmax(m2, __builtin_fmax(__builtin_fabs(v2.x), __builtin_fabs(v2.y)));
          m3 = __builtin_fmax(m3, __builtin_fmax(__builtin_fabs(v3.x), __builtin_fabs(v3.y)));
        }
        for (; c < N; c += 32) {
          const double2 v = gld2(xr + c);
          m0 = __builtin_fmax(m0, __builtin_fmax(__builtin_fabs(v.x), __builtin_fabs(v.y)));
        }
      } else {
        for (int c = c0; c < N; c += 16) m0 = __builtin_fmax(m0, __builtin_fabs(gld(xr + c)));
      }
    }
    double m = __builtin_fmax(__builtin_fmax(m0, m1), __builtin_fmax(m2, m3));
    m = group_max<16>(m);
    if (c0 == 0) {
      const int e = scale_exp(m);
      sexp[rr] = e;
      J.ea[rb * 16 + rr] = e;
    }
  }
  __syncthreads();
  const int rr = lane & 15, r = rb * 16 + rr, e = sexp[rr];
  const double* xr = J.X + (size_t)(r < R ? r : 0) * J.ldx;
  v4i* out = reinterpret_cast<v4i*>(J.A) + (size_t)rb * J.KB * S * 64 + lane;
  for (int kb = wave; kb < J.KB; kb += 4) {
    const int k0 = kb * kI8K + 16 * (lane >> 4);
    double x[16];
    if (vec && k0 + 16 <= N) {
#pragma unroll
      for (int j = 0; j < 16; j += 2) {
        const double2 v = gld2(xr + k0 + j);
        x[j] = (r < R) ? v.x : 0.0;
        x[j + 1] = (r < R) ? v.y : 0.0;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k = k0 + j;
        x[j] = (r < R && k < N) ? gld(xr + k) : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = __builtin_amdgcn_ldexp(x[j], -e);
    v4i sl[S];
    slice16<S>(x, sl);
#pragma unroll
    for (int s = 0; s < S; ++s) gst(out + ((size_t)kb * S + s) * 64, sl[s]);
  }
}

template <int S>
__global__ __launch_bounds__(256) void slice_x_kernel(SliceXList L) {
  const int j = find_job(L.boff, L.n, blockIdx.x);
  const SliceXJob J = L.job[j];
  if (*J.status & kStFatal) return;
  slice_x_body<S>(J, blockIdx.x - L.boff[j]);
}

// ---------------------------------------------------------------------------
// slices of the columns of C~: one block of 256 threads per 16 columns
// ---------------------------------------------------------------------------
__device__ __forceinline__ double c_entry(const CauchyDesc& d, int j, const ColDesc& c) {
  if (j >= d.N || c.type < 0) return 0.0;
  const RowVals rv{gld(d.rzeta + j), gld(d.rg + j), gld(d.rh + j), gld(d.rcl + j)};
  return general_entry(j, rv, c);
}

template <int S>
__device__ void slice_c_body(const SliceCJob& J, int cb) {
  __shared__ double smax[16][17];
  __shared__ int sexp[16];
  const CauchyDesc& d = J.d;
  const int N = d.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    // column maxima: thread (cc, j0) runs over rows j0, j0 + 16, ...
    const int cc = tid & 15, j0 = tid >> 4;
    const ColDesc c = load_col(d, cb * 16 + cc);
    double m = 0.0;
    for (int j = j0; j < N; j += 16) m = __builtin_fmax(m, __builtin_fabs(c_entry(d, j, c)));
    smax[cc][j0] = m;
  }
  __syncthreads();
  if (tid < 16) {
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) m = __builtin_fmax(m, smax[tid][k]);
    const int e = scale_exp(m);
    sexp[tid] = e;
    J.eb[cb * 16 + tid] = e;
  }
  __syncthreads();
  const int cc = lane & 15, e = sexp[cc];
  const ColDesc c = load_col(d, cb * 16 + cc);
  v4i* out = reinterpret_cast<v4i*>(J.B) + (size_t)cb * J.KB * S * 64 + lane;
  for (int kb = wave; kb < J.KB; kb += 4) {
    const int k0 = kb * kI8K + 16 * (lane >> 4);
    double x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = __builtin_amdgcn_ldexp(c_entry(d, k0 + j, c), -e);
    v4i sl[S];
    slice16<S>(x, sl);
#pragma unroll
    for (int s = 0; s < S; ++s) gst(out + ((size_t)kb * S + s) * 64, sl[s]);
  }
}

template <int S>
__global__ __launch_bounds__(256) void slice_c_kernel(SliceCList L) {
  const int j = find_job(L.boff, L.n, blockIdx.x);
  const SliceCJob J = L.job[j];
  if (*J.d.status & kStFatal) return;
  slice_c_body<S>(J, blockIdx.x - L.boff[j]);
}

// ---------------------------------------------------------------------------
// the product from the slices
// ---------------------------------------------------------------------------
// XCD-aware tile order. Consecutive blocks of a launch are dealt to the 8
// XCDs in turn; local tile t goes to position q of XCD t % 8's share of the
// grid, and q runs through groups of 4 tile rows column by column, so the
// blocks an XCD runs at the same time share 4 row panels of X and a few
// column panels of C~ in its L2.
__device__ __forceinline__ void i8_tile_order(int t, int tiles_m, int tiles_n, int* tm, int* tn) {
  const int tiles = tiles_m * tiles_n;
  const int full = (tiles / 8) * 8;
  const int q = (t < full) ? (t % 8) * (tiles / 8) + t / 8 : t;
  constexpr int GM = 4;
  const int per = GM * tiles_n;
  const int g = q / per, first = g * GM;
  const int gm = min(tiles_m - first, GM);
  const int w = q - g * per;
  *tm = first + w % gm;
  *tn = w / gm;
}

// A block of kI8Threads (8 waves) computes a kI8BM x kI8BN tile; wave w owns
// rows 16 w .. 16 w + 15 and all kI8BN columns, so its S x 4 accumulators take
// 112 registers and two waves fit on each SIMD: while one waits for its next
// slices the other keeps the matrix cores busy. The S slice tiles of C~ for a
// k step are staged in LDS (double-buffered, one barrier per k step); each
// wave streams its own X slices from global memory one k step ahead.
constexpr int kI8Threads = 512;

template <int S>
__global__ __launch_bounds__(kI8Threads, 1) void gemm_i8_kernel(I8List L) {
  constexpr int TILE = S * 64;          // v4i per (block, k step) group of S slice tiles
  constexpr int NBT = 4 * TILE;         // v4i of C~ slices per k step
  constexpr int NB = (NBT + kI8Threads - 1) / kI8Threads;
  static_assert(kI8BM == 16 * (kI8Threads / 64) && kI8BN == 64, "one 16-row block per wave, 4 column blocks");
  __shared__ v4i Bs[2][NBT];
  const int jb = find_job(L.boff, L.n, blockIdx.x);
  const I8Job J = L.job[jb];
  if (*J.d.status & kStFatal) return;
  int tm, tn;
  i8_tile_order(blockIdx.x - L.boff[jb], J.tiles_m, J.tiles_n, &tm, &tn);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    // a column tile of deflated columns only: copies and one reflection from
    // the FP64 X, as in the FP64 product (the LDS buffers hold the members)
    const ColDesc cc[1] = {load_col_tile(J.d, tn * kI8BN + lane)};
    int cl[1];
    const unsigned cp = copy_chunks<1>(J.d, tn * kI8BN, cc, cl);
    if (cp) {
      constexpr int SM = 2048;   // members staged per pass
      static_assert(SM * 12 + kI8BM * 8 <= (int)sizeof(Bs), "copy-path staging fits the LDS buffers");
      double* rhs = reinterpret_cast<double*>(&Bs[0][0]);
      int* js = reinterpret_cast<int*>(rhs + SM);
      double* dots = reinterpret_cast<double*>(js + SM);
      copy_path<kI8BM, kI8Threads, 1, SM>(J, tm * kI8BM, tn * kI8BN, cc, cl, cp, rhs, js, dots);
      return;
    }
  }
  const int KB = J.KB;
  const v4i* A = reinterpret_cast<const v4i*>(J.A);
  const v4i* B = reinterpret_cast<const v4i*>(J.B);
  const int rb = tm * (kI8BM / 16) + wave, cb0 = tn * (kI8BN / 16);
  const v4i* ap = A + (size_t)rb * KB * TILE + lane;
  // this thread's share of the block's C~ fragments: elements tid + kI8Threads i
  // of the NBT of a k step (column block c = e / TILE, offset e % TILE)
  const v4i* bp[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = min(tid + kI8Threads * i, NBT - 1), c = e / TILE;
    bp[i] = B + (size_t)(cb0 + c) * KB * TILE + (e - c * TILE);
  }

  v4i acc[S][4];
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[g][c] = v4i{0, 0, 0, 0};

  // The loads of step kb + 1 are issued right after the barrier of step kb and
  // consumed at the top of step kb + 1, so no wait for them falls inside the
  // MFMA sequence (nor for the first step's loads, issued the same way).
  v4i a[S], an[S], bn[NB];
  auto load_next = [&](int kb) {
    const size_t o = (size_t)kb * TILE;
#pragma unroll
    for (int s = 0; s < S; ++s) an[s] = gld(ap + o + s * 64);
#pragma unroll
    for (int i = 0; i < NB; ++i) bn[i] = gld(bp[i] + o);
  };
  load_next(0);
  for (int kb = 0; kb < KB; ++kb) {
    v4i* Bc = Bs[kb & 1];
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (NBT % kI8Threads == 0 || tid + kI8Threads * i < NBT) Bc[tid + kI8Threads * i] = bn[i];
#pragma unroll
    for (int s = 0; s < S; ++s) a[s] = an[s];
    __syncthreads();
    if (kb + 1 < KB) load_next(kb + 1);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      v4i b[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bc[(c * S + t) * 64 + lane];
#pragma unroll
      for (int s = 0; s + t < S; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[s + t][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], b[c], acc[s + t][c], 0, 0, 0);
    }
  }

  // epilogue: sum_g acc_g 2^(-7 g) by Horner in FP64, times 2^(Ex + Ec - 12)
  const int row0 = tm * kI8BM + 16 * wave + 4 * (lane >> 4);
  const int colx = tn * kI8BN + (lane & 15);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = colx + 16 * c;
    if (col >= J.N) continue;
    const int ec = gld(J.eb + col) - 12;
    const double sc = J.d.colscale ? gld(J.d.colscale + col) : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + v;
      if (row >= J.R) continue;
      double x = (double)acc[S - 1][c][v];
#pragma unroll
      for (int g = S - 2; g >= 0; --g) x = __builtin_fma(x, 0x1p-7, (double)acc[g][c][v]);
      gst(J.Xo + (size_t)row * J.ldo + col, sc * __builtin_amdgcn_ldexp(x, gld(J.ea + row) + ec));
    }
  }
}

}  // namespace

void launch_slice_x(const SliceXList& L, int S, hipStream_t st) {
  if (L.n <= 0 || L.blocks <= 0) return;
  switch (S) {
    case 6: hipLaunchKernelGGL(slice_x_kernel<6>, dim3(L.blocks), dim3(256), 0, st, L); break;
    case 8: hipLaunchKernelGGL(slice_x_kernel<8>, dim3(L.blocks), dim3(256), 0, st, L); break;
    default: hipLaunchKernelGGL(slice_x_kernel<7>, dim3(L.blocks), dim3(256), 0, st, L); break;
  }
}

void launch_slice_c(const SliceCList& L, int S, hipStream_t st) {
  if (L.n <= 0 || L.blocks <= 0) return;
  switch (S) {
    case 6: hipLaunchKernelGGL(slice_c_kernel<6>, dim3(L.blocks), dim3(256), 0, st, L); break;
    case 8: hipLaunchKernelGGL(slice_c_kernel<8>, dim3(L.blocks), dim3(256), 0, st, L); break;
    default: hipLaunchKernelGGL(slice_c_kernel<7>, dim3(L.blocks), dim3(256), 0, st, L); break;
  }
}

void launch_gemm_i8(const I8List& L, int S, hipStream_t st) {
  if (L.n <= 0 || L.blocks <= 0) return;
  switch (S) {
    case 6: hipLaunchKernelGGL(gemm_i8_kernel<6>, dim3(L.blocks), dim3(kI8Threads), 0, st, L); break;
    case 8: hipLaunchKernelGGL(gemm_i8_kernel<8>, dim3(L.blocks), dim3(kI8Threads), 0, st, L); break;
    default: hipLaunchKernelGGL(gemm_i8_kernel<7>, dim3(L.blocks), dim3(kI8Threads), 0, st, L); break;
  }
}

}  // namespace svdu
