// Job tables. Every launch of libsvdu serves a list of independent jobs: the
// eigen-updates, products or projections of one rank-1 update, or of many
// updates batched together. Job i of a list owns blocks [boff[i], boff[i+1])
// of the launch and a block finds its job by a binary search over boff (a
// uniform loop over scalar loads). A job's arithmetic does not depend on the
// other jobs of its list, so a result is the same alone and batched.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "svdu_internal.h"

namespace svdu {

// Largest i < n with boff[i] <= b (jobs with no blocks are skipped).
__device__ __forceinline__ int find_job(const int* __restrict__ boff, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boff[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Vectors carried through C~^T after an eigen-update: y_k = C~^T x_k, k < nv
// (nv = 0: none).
struct TmvJob {
  int nv;
  const double* x[3];
  double* y[3];
};

// The eigen-updates of one level (the first or the second update of each
// side of every rank-1 update in the launch), with the block offsets of the
// three launch shapes used by the stage kernels: one block per job
// (deflation), one wave per root or pole (4 per block), one thread per index
// (256 per block).
// The kernels that sum over all K poles or roots for each of K items (secular
// roots, Loewner weights, column norms, transposed Cauchy products) give each
// item a group of kSmallGroup lanes for eigenproblems up to order kGroupMaxN
// (short sums: fewer lanes per item waste less on reductions and per-item
// logic, yet one problem alone still spreads over many waves) and a whole
// wave above it. The choice depends on the order alone, so a problem gets
// the same arithmetic alone and in a batch.
constexpr int kGroupMaxN = 2048;
constexpr int kSmallGroup = 16;
// Poles per leaf of the far-field form of the secular solve (one block per leaf).
constexpr int kSfLeaf = 64;

struct StageLevel {
  int n = 0;
  const Stage* st = nullptr;
  const TmvJob* tmv = nullptr;   // n entries, or nullptr
  const int* boff_w = nullptr;   // ceil(N / 4) blocks per job
  const int* boff_t = nullptr;   // ceil(N / 256) blocks per job
  const int* boff_i = nullptr;   // item kernels: ceil(N / (256 / kSmallGroup)) if N <= kGroupMaxN, else ceil(N / 4)
  const int* boff_s = nullptr;   // secular kernel: ceil(item blocks / 4) blocks of 1024 threads per job
  const int* boff_l = nullptr;   // far-field secular kernel: ceil(N / kSfLeaf) + 1 blocks per job
  int blocks_w = 0, blocks_t = 0, blocks_i = 0, blocks_s = 0, blocks_l = 0;
  int nmax = 0;                  // largest order of the level (host side)
};

// One product X_out = X C~ in the tile grid of the list's tile shape.
struct GemmJob {
  int R, ldx, ldo, vec_a;
  int shape, tiles_n, tiles;
  const double* X;
  double* Xo;
  CauchyDesc d;
};

struct GemmList {
  int n = 0;
  int blocks = 0;               // total tiles
  const int* boff = nullptr;
  const GemmJob* job = nullptr;
  int* counter = nullptr;       // persistent schedule: next tile (zeroed before the launch)
  int copy = 0;                 // some job carries cluster members (FP64 copy-path kernels)
};

// X^T [v0 v1 v2] for X row-major R x N, in column blocks x row chunks.
struct GemvJob {
  int R, N, ldx, nv, cblocks, chunks;
  const double* X;
  const double* v[3];
  double* out[3];
  double* part;
};

struct GemvList {
  int n = 0;
  int blocks_p = 0, blocks_r = 0;
  const int* boff_p = nullptr;  // partial sums: cblocks * chunks blocks per job
  const int* boff_r = nullptr;  // reduction: ceil(nv N / 256) blocks per job
  const GemvJob* job = nullptr;
};

// Column renormalisation of one factor (precision form).
struct RenormJob {
  int R, N, ld, cblocks, chunks;
  double* X;
  double* part;
  const int* status;
};

struct RenormList {
  int n = 0;
  int blocks = 0;
  const int* boff = nullptr;    // cblocks * chunks per job
  const RenormJob* job = nullptr;
};

// Refinement of close singular-value clusters of one update (k_refine.hip).
struct RefineJob {
  int m, n, kmax, cmax;            // cmax: cluster records, kmax: gathered columns
  const double *U, *V, *a, *b, *sigma;
  int ldu, ldv;
  double *Uo, *so, *Vo;            // the update's outputs, refined in place
  int lduo, ldvo;
  const int* status;
  int* info;                       // [0] gathered columns k, [1] clusters
  int *cl_start, *cl_size, *cl_off, *col_idx;
  double *Yu, *Yv, *T, *W, *beta;  // kmax x m, kmax x n, kmax x m, kmax x m, kmax
};

struct RefineList {
  int n = 0;
  int blocks_n = 0, blocks_c = 0, blocks_w = 0, blocks_cl = 0;
  const int* boff_n = nullptr;     // ceil(n / 256) per update (gather)
  const int* boff_c = nullptr;     // ceil((m + 1) / 16) per update (V^T products)
  const int* boff_w = nullptr;     // ceil(m / 4) per update (U products)
  const int* boff_cl = nullptr;    // blocks sharing the clusters of an update
  const RefineJob* job = nullptr;
};

// ---- exact-slice INT8 product (precision form SVDU_PREC_SLICED_INT8) ------------
// X (R x N, FP64) and C~ (N x N) are each split into S signed 7-bit slices
// with a power-of-two scale per row of X and per column of C~; the slices sit
// in HBM as 1 KiB tiles of 16 rows (or columns) x 64 k, one tile per slice,
// each tile in the operand order of v_mfma_i32_16x16x64_i8 (lane l holds row
// l % 16, k = 16 (l / 16) .. + 15). Rows are padded with zero slices to a
// multiple of kI8BM, columns to kI8BN and k to 64.
constexpr int kI8BM = 128, kI8BN = 64, kI8K = 64;
constexpr int kMinSlices = 6, kMaxSlices = 8, kDefaultSlices = 7;
// Largest order for the INT8 form: a group of S <= 8 slice dot products over N
// terms of at most 64^2 stays below 2^31.
constexpr int kI8MaxN = 32768;
__host__ __device__ constexpr int i8_pad(int x, int q) { return (x + q - 1) / q * q; }

// Slices of the rows of X: A tile (rb, kb, s) at A + ((rb * KB + kb) * S + s) * 1024.
struct SliceXJob {
  int R, N, ldx, KB, rblocks;   // rblocks = padded rows / 16
  const double* X;
  int8_t* A;
  int* ea;                      // per padded row: exponent of its scale
  const int* status;
};
// Slices of the columns of C~: B tile (cb, kb, s) at B + ((cb * KB + kb) * S + s) * 1024.
struct SliceCJob {
  CauchyDesc d;                 // N = d.N
  int KB, cblocks;              // cblocks = padded columns / 16
  int8_t* B;
  int* eb;                      // per padded column
};
// X_out = X C~ from the slices, in tiles of kI8BM x kI8BN. Column tiles made
// only of deflated columns (the zero block of a rectangular problem) are
// written from the FP64 X by the copy path instead (copy_path.h).
struct I8Job {
  int R, N, ldo, KB, tiles_m, tiles_n, tiles;
  const int8_t* A;
  const int8_t* B;
  const int* ea;
  const int* eb;
  double* Xo;
  const double* X;              // the FP64 X, for the copy path
  int ldx;
  CauchyDesc d;                 // C~ (colscale: optional per-column sign; members when n > m)
};

struct SliceXList {
  int n = 0, blocks = 0;
  const int* boff = nullptr;    // rblocks per job
  const SliceXJob* job = nullptr;
};
struct SliceCList {
  int n = 0, blocks = 0;
  const int* boff = nullptr;    // cblocks per job
  const SliceCJob* job = nullptr;
};
struct I8List {
  int n = 0, blocks = 0;
  const int* boff = nullptr;    // tiles per job
  const I8Job* job = nullptr;
};

// Slices every job's X / C~, then the products from the slices (S slices).
void launch_slice_x(const SliceXList& L, int S, hipStream_t st);
void launch_slice_c(const SliceCList& L, int S, hipStream_t st);
void launch_gemm_i8(const I8List& L, int S, hipStream_t st);

// ---- launchers (each enqueues on `st`, no host synchronisation) ----------------
// Projections of every GemvJob: partial sums per row chunk, then a
// fixed-order reduction.
void launch_gemv_list(const GemvList& L, hipStream_t st);
int gemv_cblocks(int N);
int gemv_chunks(int R);
size_t gemv_t_scratch_elems(int R, int N, int nv);
// Deflation, secular roots, Loewner weights, column norms, descriptors of
// every eigen-update of a level.
// far_field (SVDU_OPT_SECULAR_FMM): 0 the secular roots from the direct sums;
// 1 with the far field from per-leaf interpolants for orders above
// kGroupMaxN; 2 with it at every order.
void launch_stage_level(const StageLevel& L, int maxit, int far_field, hipStream_t st);
// The secular solve alone (svdu_secular).
void launch_secular_level(const StageLevel& L, int maxit, int far_field, hipStream_t st);
// y = C~^T x for the TmvJobs of a level.
void launch_cauchy_tmatvec_level(const StageLevel& L, hipStream_t st);
// X_out = X C~ for every job of the list, in tile shape `shape` (TileShape),
// one block per tile (grid) or at most grid_cap blocks taking tiles from
// L.counter (persistent).
void launch_gemm_f64(const GemmList& L, int shape, bool persistent, int grid_cap, hipStream_t st);
void launch_gemm_split32(const GemmList& L, int shape, bool persistent, int grid_cap, hipStream_t st);
// Column renormalisation of every RenormJob; scratch per job >=
// renorm_scratch_elems(R, N) doubles.
void launch_column_renorm(const RenormList& L, hipStream_t st);
// Cluster refinement of every update of the list.
void launch_refine(const RefineList& L, hipStream_t st);
size_t renorm_scratch_elems(int R, int N);

}  // namespace svdu
