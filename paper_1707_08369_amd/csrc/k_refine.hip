// Refinement of close singular-value clusters (not in the paper).
//
// The method computes the left vectors from A^ A^T and the right vectors from
// A^T A^ independently. Inside a group of relatively close singular values
// each side's eigenvectors are accurate to about u / relgap within the group's
// span, and the two sides' errors do not match, so U^ S^ V^^T misses A^ by
// about sigma u / relgap in that block. For every cluster of consecutive
// sigma^ with relative gaps (sigma_i - sigma_{i+1}) / sigma_i <= tau (and sigma^
// not negligible against sigma^_0), this pass forms the small block
// B = U^_c^T A^ V^_c from the inputs,
//   A^ V^_c = U (S (V^T V^_c)) + a (b^T V^_c),
// takes its SVD B = P diag(s) Q^T (one-sided Jacobi, s descending), and
// replaces U^_c and V^_c by U^_c P and V^_c Q. sigma^ itself is kept (it is
// the secular solution; s differs from it by O(u |A^|)), so singular values
// and deflation are not touched. Work: one pass over V and one over U per
// kRefineChunk gathered columns (at most kmax), and O(m) per block entry.
#include <math.h>

#include "device_util.h"
#include "jobs.h"
#include "svdu_internal.h"

namespace svdu {

constexpr double kRefineTau = 1e-6;   // relative gap below which neighbours are refined together
constexpr int kRefineSmax = 8;        // largest cluster refined as one block
constexpr int kRefineChunk = 8;       // gathered columns per pass of the skinny products

// ---------------------------------------------------------------------------
// cluster detection: one block per update. A thread whose sigma^ index starts a
// run of close neighbours walks the run and cuts it into clusters of at most
// kRefineSmax; block scans give every cluster its record and column offset.
// Columns beyond kmax are not refined (sigma^ descending: the largest first).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool refine_link(const double* so, int m, double tiny, double tau, int i) {
  if (i < 0 || i >= m - 1) return false;
  const double a = so[i], b = so[i + 1];
  if (!(a > tiny)) return false;
  return a - b <= tau * a;
}

__global__ __launch_bounds__(256) void refine_detect_kernel(RefineList L) {
  __shared__ int shi[64];
  __shared__ int first_skip;
  const RefineJob J = L.job[blockIdx.x];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (*J.status & kStFatal) {
    if (tid == 0) J.info[0] = J.info[1] = 0;
    return;
  }
  const int m = J.m;
  const double s0 = J.so[0];
  const double tiny = 64.0 * kU * s0, lim = kRefineTau;
  if (tid == 0) first_skip = 1 << 30;
  __syncthreads();
  int carry_c = 0, carry_cols = 0;
  for (int base = 0; base < m; base += nt) {
    const int i = base + tid;
    const bool start = refine_link(J.so, m, tiny, lim, i) && !refine_link(J.so, m, tiny, lim, i - 1);
    // walk: count clusters and columns of the run starting at i
    int nc = 0, ncol = 0;
    if (start) {
      int j = i;
      while (true) {
        int s = 1;
        while (s < kRefineSmax && refine_link(J.so, m, tiny, lim, j + s - 1)) ++s;
        ++nc;
        ncol += s;
        if (!refine_link(J.so, m, tiny, lim, j + s - 1)) break;
        j += s;
      }
    }
    int tot_c, tot_cols;
    const int ex_c = block_scan_incl(nc, shi, &tot_c) - nc;
    const int ex_col = block_scan_incl(ncol, shi, &tot_cols) - ncol;
    if (start) {
      int j = i, c = carry_c + ex_c, off = carry_cols + ex_col;
      while (true) {
        int s = 1;
        while (s < kRefineSmax && refine_link(J.so, m, tiny, lim, j + s - 1)) ++s;
        if (c < J.cmax) {
          J.cl_start[c] = j;
          J.cl_off[c] = off;
          if (off + s <= J.kmax) {
            J.cl_size[c] = s;
            for (int q = 0; q < s; ++q) J.col_idx[off + q] = j + q;
          } else {
            J.cl_size[c] = 0;
            atomicMin(&first_skip, off);
          }
        } else {
          atomicMin(&first_skip, off);
        }
        ++c;
        off += s;
        if (!refine_link(J.so, m, tiny, lim, j + s - 1)) break;
        j += s;
      }
    }
    carry_c += tot_c;
    carry_cols += tot_cols;
  }
  __syncthreads();
  if (tid == 0) {
    const int k = carry_cols < first_skip ? carry_cols : first_skip;
    J.info[0] = k < J.kmax ? k : J.kmax;
    J.info[1] = carry_c < J.cmax ? carry_c : J.cmax;
  }
}

// ---------------------------------------------------------------------------
// gather the cluster columns of U^ and V^ (contiguous per column)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void refine_gather_kernel(RefineList L) {
  const int u = find_job(L.boff_n, L.n, blockIdx.x);
  const RefineJob J = L.job[u];
  const int k = J.info[0];
  const int r = (blockIdx.x - L.boff_n[u]) * 256 + threadIdx.x;
  if (k <= 0 || r >= J.n) return;
  for (int q = 0; q < k; ++q) {
    const int c = J.col_idx[q];
    J.Yv[(size_t)q * J.n + r] = J.Vo[(size_t)r * J.ldvo + c];
    if (r < J.m) J.Yu[(size_t)q * J.m + r] = J.Uo[(size_t)r * J.lduo + c];
  }
}

// ---------------------------------------------------------------------------
// T[q][j] = sigma_j sum_r Yv[q][r] V[r][j] for j < m, and beta[q] = sum_r Yv[q][r] b[r]
// (j = m): one pass over V for all k gathered columns, on the matrix cores.
// Block: 16 columns of [V b] and all n rows; its 4 waves take interleaved
// 4-row steps and are summed in a fixed order at the end. A operand: 16
// gathered columns (lane l: Yv[16 qb + l % 16][r + l / 16]); B operand: lane l
// holds V[r + l / 16][j0 + l % 16]; result register v of lane l holds
// T[16 qb + l / 16 + 4 v][j0 + l % 16]. Rows q >= k read row k - 1 and rows
// r >= n carry a zero B entry, so neither reaches a stored result.
// ---------------------------------------------------------------------------
typedef double rf4 __attribute__((ext_vector_type(4)));
constexpr int kVtCols = 16;
constexpr int kVtMaxQb = 8;   // 16-column groups of the gathered columns (kmax <= 128)

template <int KB>
__device__ void refine_vt_body(const RefineJob& J, int k, int j0, rf4 (*red)[kVtMaxQb][64]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  const int j = j0 + i, jc = min(j, J.m - 1);
  const double* yrow[KB];
#pragma unroll
  for (int qb = 0; qb < KB; ++qb) yrow[qb] = J.Yv + (size_t)min(16 * qb + i, k - 1) * J.n;
  rf4 acc[KB];
#pragma unroll
  for (int qb = 0; qb < KB; ++qb) acc[qb] = rf4{0.0, 0.0, 0.0, 0.0};
  const int nsteps = (J.n + 3) / 4;
  for (int st = wv; st < nsteps; st += 4) {
    const int r = 4 * st + kq, rc = min(r, J.n - 1);
    const double vv = gld(J.V + (size_t)rc * J.ldv + jc), bb = gld(J.b + rc);
    const double bv = (r < J.n) ? (j < J.m ? vv : (j == J.m ? bb : 0.0)) : 0.0;
#pragma unroll
    for (int qb = 0; qb < KB; ++qb)
      acc[qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(gld(yrow[qb] + rc), bv, acc[qb], 0, 0, 0);
  }
#pragma unroll
  for (int qb = 0; qb < KB; ++qb) red[wv][qb][lane] = acc[qb];
  __syncthreads();
  for (int e = threadIdx.x; e < KB * 4 * 64; e += blockDim.x) {
    const int qb = e >> 8, v = (e >> 6) & 3, l = e & 63;
    const int q = 16 * qb + (l >> 4) + 4 * v, jj = j0 + (l & 15);
    if (q >= k || jj > J.m) continue;
    const double t = ((red[0][qb][l][v] + red[1][qb][l][v]) + red[2][qb][l][v]) + red[3][qb][l][v];
    if (jj < J.m)
      J.T[(size_t)q * J.m + jj] = J.sigma[jj] * t;   // S V^T v^
    else
      J.beta[q] = t;
  }
}

__global__ __launch_bounds__(256) void refine_vt_kernel(RefineList L) {
  __shared__ rf4 red[4][kVtMaxQb][64];
  const int u = find_job(L.boff_c, L.n, blockIdx.x);
  const RefineJob J = L.job[u];
  const int k = J.info[0];
  if (k <= 0) return;
  const int j0 = (blockIdx.x - L.boff_c[u]) * kVtCols;
  switch ((k + 15) / 16) {
    case 1: refine_vt_body<1>(J, k, j0, red); break;
    case 2: refine_vt_body<2>(J, k, j0, red); break;
    case 3: refine_vt_body<3>(J, k, j0, red); break;
    case 4: refine_vt_body<4>(J, k, j0, red); break;
    case 5: refine_vt_body<5>(J, k, j0, red); break;
    case 6: refine_vt_body<6>(J, k, j0, red); break;
    case 7: refine_vt_body<7>(J, k, j0, red); break;
    default: refine_vt_body<8>(J, k, j0, red); break;
  }
}

// ---------------------------------------------------------------------------
// W[q][r] = sum_j U[r][j] T[q][j] + a[r] beta[q]: one wave per row of U.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void refine_u_kernel(RefineList L) {
  const int u = find_job(L.boff_w, L.n, blockIdx.x);
  const RefineJob J = L.job[u];
  const int k = J.info[0];
  if (k <= 0) return;
  const int lane = threadIdx.x & 63;
  const int r = (blockIdx.x - L.boff_w[u]) * 4 + (threadIdx.x >> 6);
  if (r >= J.m) return;
  const double* ur = J.U + (size_t)r * J.ldu;
  for (int q0 = 0; q0 < k; q0 += kRefineChunk) {
    double acc[kRefineChunk];
#pragma unroll
    for (int v = 0; v < kRefineChunk; ++v) acc[v] = 0.0;
    for (int jj = lane; jj < J.m; jj += 64) {
      const double x = ur[jj];
#pragma unroll
      for (int v = 0; v < kRefineChunk; ++v)
        if (q0 + v < k) acc[v] += x * J.T[(size_t)(q0 + v) * J.m + jj];
    }
#pragma unroll
    for (int v = 0; v < kRefineChunk; ++v) {
      const double t = wave_sum(acc[v]);
      if (lane == 0 && q0 + v < k) J.W[(size_t)(q0 + v) * J.m + r] = t + J.a[r] * J.beta[q0 + v];
    }
  }
}

// ---------------------------------------------------------------------------
// Per cluster: B = Yu^T W (s x s), its SVD by one-sided Jacobi (thread 0),
// then U^_c <- Yu P, V^_c <- Yv Q (singular values descending).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void refine_apply_kernel(RefineList L) {
  constexpr int S = kRefineSmax;
  __shared__ double B[S][S], P[S][S], Q[S][S], sv[S];
  __shared__ double sh[64];
  const int u = find_job(L.boff_cl, L.n, blockIdx.x);
  const RefineJob J = L.job[u];
  const int ncl = J.info[1];
  const int tid = threadIdx.x;
  const int per = L.boff_cl[u + 1] - L.boff_cl[u];
  for (int c = blockIdx.x - L.boff_cl[u]; c < ncl; c += per) {
    const int s = J.cl_size[c];
    if (s < 2) continue;   // uniform across the block
    const int off = J.cl_off[c];
    for (int i = 0; i < s; ++i)
      for (int j2 = 0; j2 < s; ++j2) {
        double d = 0.0;
        for (int r = tid; r < J.m; r += blockDim.x)
          d += J.Yu[(size_t)(off + i) * J.m + r] * J.W[(size_t)(off + j2) * J.m + r];
        d = block_sum(d, sh);
        if (tid == 0) B[i][j2] = d;
      }
    __syncthreads();
    if (tid == 0) {
      // one-sided Jacobi on the columns of B: B Q = P diag(sv)
      for (int i = 0; i < s; ++i)
        for (int j2 = 0; j2 < s; ++j2) Q[i][j2] = (i == j2) ? 1.0 : 0.0;
      for (int sweep = 0; sweep < 30; ++sweep) {
        bool rot = false;
        for (int p = 0; p < s - 1; ++p)
          for (int q = p + 1; q < s; ++q) {
            double al = 0.0, be = 0.0, ga = 0.0;
            for (int i = 0; i < s; ++i) {
              al += B[i][p] * B[i][p];
              be += B[i][q] * B[i][q];
              ga += B[i][p] * B[i][q];
            }
            if (fabs(ga) <= 1e-17 * sqrt(al * be) || ga == 0.0) continue;
            rot = true;
            const double zeta = (be - al) / (2.0 * ga);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
            for (int i = 0; i < s; ++i) {
              const double bp = B[i][p], bq = B[i][q];
              B[i][p] = cs * bp - sn * bq;
              B[i][q] = sn * bp + cs * bq;
              const double qp = Q[i][p], qq = Q[i][q];
              Q[i][p] = cs * qp - sn * qq;
              Q[i][q] = sn * qp + cs * qq;
            }
          }
        if (!rot) break;
      }
      // singular values, left vectors, descending order
      int ord[S];
      for (int j2 = 0; j2 < s; ++j2) {
        double nn = 0.0;
        for (int i = 0; i < s; ++i) nn += B[i][j2] * B[i][j2];
        sv[j2] = sqrt(nn);
        ord[j2] = j2;
      }
      for (int a = 1; a < s; ++a)
        for (int b2 = a; b2 > 0 && sv[ord[b2]] > sv[ord[b2 - 1]]; --b2) {
          const int t = ord[b2];
          ord[b2] = ord[b2 - 1];
          ord[b2 - 1] = t;
        }
      double Pt[S][S], Qt[S][S], st[S];
      for (int j2 = 0; j2 < s; ++j2) {
        const int o = ord[j2];
        st[j2] = sv[o];
        for (int i = 0; i < s; ++i) {
          Pt[i][j2] = (sv[o] > 0.0) ? B[i][o] / sv[o] : ((i == o) ? 1.0 : 0.0);
          Qt[i][j2] = Q[i][o];
        }
      }
      for (int j2 = 0; j2 < s; ++j2) {
        sv[j2] = st[j2];
        for (int i = 0; i < s; ++i) {
          P[i][j2] = Pt[i][j2];
          Q[i][j2] = Qt[i][j2];
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < J.n; r += blockDim.x) {
      double yv[S], yu[S];
      for (int i = 0; i < s; ++i) {
        yv[i] = J.Yv[(size_t)(off + i) * J.n + r];
        yu[i] = (r < J.m) ? J.Yu[(size_t)(off + i) * J.m + r] : 0.0;
      }
      for (int j2 = 0; j2 < s; ++j2) {
        double nv = 0.0, nu = 0.0;
        for (int i = 0; i < s; ++i) {
          nv += yv[i] * Q[i][j2];
          nu += yu[i] * P[i][j2];
        }
        const int col = J.col_idx[off + j2];
        J.Vo[(size_t)r * J.ldvo + col] = nv;
        if (r < J.m) J.Uo[(size_t)r * J.lduo + col] = nu;
      }
    }
    __syncthreads();
  }
}

void launch_refine(const RefineList& L, hipStream_t st) {
  if (L.n <= 0) return;
  hipLaunchKernelGGL(refine_detect_kernel, dim3(L.n), dim3(256), 0, st, L);
  hipLaunchKernelGGL(refine_gather_kernel, dim3(L.blocks_n), dim3(256), 0, st, L);
  hipLaunchKernelGGL(refine_vt_kernel, dim3(L.blocks_c), dim3(256), 0, st, L);
  hipLaunchKernelGGL(refine_u_kernel, dim3(L.blocks_w), dim3(256), 0, st, L);
  hipLaunchKernelGGL(refine_apply_kernel, dim3(L.blocks_cl), dim3(256), 0, st, L);
}

}  // namespace svdu
