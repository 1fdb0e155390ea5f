// C ABI of libsvdu: argument checks, workspace layout and the order of the
// device work for one rank-1 SVD update (Section 6.1 of the paper).
//
// Device work, all on the caller's stream:
//   1. probes w1, w2 and the status word;
//   2. projections p = U^T a, [q t1 t2] = V^T [b w1 w2] (one pass over each of
//      U and V, Algorithm Step 1 / RankOneUpdate Step 1);
//   3. the 2x2 splits (Algorithm Steps 2-3) and every projected vector in core
//      space: U^T a1 = q11 p + q21 S q, U^T b1 = q12 p + q22 S q, and the same
//      on the right with S^T p; validation of the inputs;
//   4. the four eigen-updates (Steps 4-7): deflation, secular roots, weights,
//      descriptors of C~; the second update of each side gets its z as
//      C~^T (U^T b1) of the first;
//   5. singular values (Step 8) and the signs that pair V^ with U^ (not in
//      the paper): s_i = sign((U^T A^ w)_i (V^T w)_i) from two probes mapped
//      through the C~^T of both updates;
//   6. the four products X C~ (Steps 4-7), FP64 MFMA.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/svdu.h"
#include "device_util.h"
#include "fmm_plan.h"
#include "svdu_internal.h"

namespace svdu {
namespace {

int g_maxit = 200;

// Timing ring: when enabled, each svdu_rank1_update records HIP events on the
// caller's stream at the boundaries of its phases (projections | O(n^2)
// eigen-update work | product L+ | product L- | product R+ | product R- |
// flags), for up to kRingCalls calls. Host-side only; events are created once.
constexpr int kRingCalls = 256, kRingEvents = 8;
struct TimingRing {
  bool on = false;
  int count = 0;
  bool made[kRingCalls] = {};
  hipEvent_t ev[kRingCalls][kRingEvents];
};
TimingRing g_ring;

int ring_begin() {
  if (!g_ring.on || g_ring.count >= kRingCalls) return -1;
  const int c = g_ring.count;
  if (!g_ring.made[c]) {
    for (int k = 0; k < kRingEvents; ++k)
      if (hipEventCreate(&g_ring.ev[c][k]) != hipSuccess) return -1;
    g_ring.made[c] = true;
  }
  ++g_ring.count;
  return c;
}
void ring_mark(int call, int k, hipStream_t st) {
  if (call >= 0) (void)hipEventRecord(g_ring.ev[call][k], st);
}

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

void carve_stage(Carver& c, Stage& s, int cap) {
  const size_t n = cap > 0 ? cap : 1;
  s.cap = cap;
  s.rho = c.take<double>(1);
  s.dsort = c.take<double>(n);
  s.zs = c.take<double>(n);
  s.clu = c.take<int>(n);
  s.Llist = c.take<int>(n);
  s.g = c.take<double>(n);
  s.W = c.take<double>(n);
  s.W2 = c.take<double>(n);
  s.cfirst = c.take<int>(n);
  s.csize = c.take<int>(n);
  s.dlist = c.take<int>(n);
  s.dval = c.take<double>(n);
  s.counts = c.take<int>(4);
  s.org = c.take<int>(n);
  s.tau = c.take<double>(n);
  s.mu = c.take<double>(n);
  s.what = c.take<double>(n);
  s.cs = c.take<double>(n);
  s.iters = c.take<int>(n);
  s.rg = c.take<double>(n);
  s.rzeta = c.take<double>(n);
  s.rh = c.take<double>(n);
  s.rcl = c.take<int>(n);
  s.flags = c.take<int8_t>(n);
  s.ctype = c.take<int8_t>(n);
  s.co = c.take<double>(n);
  s.ctau = c.take<double>(n);
  s.ccs = c.take<double>(n);
  s.ccl = c.take<int>(n);
  s.cmem = c.take<int>(n);
  s.ch = c.take<double>(n);
  s.lam_out = c.take<double>(n);
  s.hx = c.take<double>(3 * n);
  s.col_of = c.take<int>(n);
  s.rootpos = c.take<int>(n);
  s.dpos = c.take<int>(n);
}

// Everything svdu_rank1_update keeps in the workspace.
struct Layout {
  int* status;
  double* scal;  // [0] beta [1] alpha [2] b.w1 [3] b.w2
  double *p, *q, *t1, *t2, *w1, *w2;
  double *zLp, *yLm, *pL1, *pL2, *zLm, *pL1b, *pL2b, *fL1, *fL2;
  double *zRp, *yRm, *zRm, *pR1b, *pR2b, *fR1, *fR2;
  double *lamLp, *lamRp, *signs;
  double* gemv_scratch;
  size_t gemv_elems;
  double* renorm_scratch;
  double* T;  // n x n intermediate basis
  Stage st[4];
  double* fmm_work;     // FMM path only
  size_t fmm_elems;
  char* fmm_plan;
  size_t fmm_plan_bytes;
  size_t bytes;
};

Layout carve_update(void* base, int m, int n, int path) {
  Layout L;
  Carver c(base);
  L.status = c.take<int>(16);
  L.scal = c.take<double>(8);
  L.p = c.take<double>(m);
  L.q = c.take<double>(n);
  L.t1 = c.take<double>(n);
  L.t2 = c.take<double>(n);
  L.w1 = c.take<double>(n);
  L.w2 = c.take<double>(n);
  L.zLp = c.take<double>(m);
  L.yLm = c.take<double>(m);
  L.pL1 = c.take<double>(m);
  L.pL2 = c.take<double>(m);
  L.zLm = c.take<double>(m);
  L.pL1b = c.take<double>(m);
  L.pL2b = c.take<double>(m);
  L.fL1 = c.take<double>(m);
  L.fL2 = c.take<double>(m);
  L.zRp = c.take<double>(n);
  L.yRm = c.take<double>(n);
  L.zRm = c.take<double>(n);
  L.pR1b = c.take<double>(n);
  L.pR2b = c.take<double>(n);
  L.fR1 = c.take<double>(n);
  L.fR2 = c.take<double>(n);
  L.lamLp = c.take<double>(m);
  L.lamRp = c.take<double>(n);
  L.signs = c.take<double>(n);
  L.gemv_elems = std::max(gemv_t_scratch_elems(m, m, 1), gemv_t_scratch_elems(n, n, 3));
  L.gemv_scratch = c.take<double>(L.gemv_elems);
  L.renorm_scratch = c.take<double>(std::max(renorm_scratch_elems(m, m), renorm_scratch_elems(n, n)));
  for (int k = 0; k < 4; ++k) carve_stage(c, L.st[k], k < 2 ? m : n);
  L.T = c.take<double>((size_t)n * n);
  L.fmm_elems = (path == SVDU_PATH_FMM) ? fmm_workspace_elems(n, n) : 0;
  L.fmm_work = c.take<double>(L.fmm_elems);
  L.fmm_plan_bytes = (path == SVDU_PATH_FMM) ? 4 * fmm_plan_bytes(n) : 0;
  L.fmm_plan = c.take<char>(L.fmm_plan_bytes);
  L.bytes = c.off + 256;
  return L;
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ void init_kernel(int n, int* status, double* w1, double* w2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) status[0] = 0;
  if (j < n) {
    w1[j] = hash_unit((uint64_t)j, 1);
    w2[j] = hash_unit((uint64_t)j, 2);
  }
}

__device__ inline void gram_split_dev(double beta, double* rp, double* rm, double Q[4]) {
  // [[beta, 1], [1, 0]] = Q diag(rp, rm) Q^T; rp rm = -1; eigenvector of r ~ (r, 1).
  const double s = hypot(beta, 2.0);
  if (beta >= 0.0) {
    *rp = 0.5 * (beta + s);
    *rm = -1.0 / *rp;
  } else {
    *rm = 0.5 * (beta - s);
    *rp = -1.0 / *rm;
  }
  const double np = hypot(*rp, 1.0), nm = hypot(*rm, 1.0);
  Q[0] = *rp / np;  // Q00
  Q[1] = *rm / nm;  // Q01
  Q[2] = 1.0 / np;  // Q10
  Q[3] = 1.0 / nm;  // Q11
}

struct SetupArgs {
  int m, n;
  const double *sigma, *a, *b, *p, *q, *t1, *t2, *w1, *w2;
  double* scal;
  int* status;
  double *rho1, *rho2, *rho3, *rho4;
  double *zLp, *yLm, *pL1, *pL2, *lamLp;
  double *zRp, *yRm, *lamRp;
  int *colLp, *colLm, *colRp, *colRm;
};

__global__ __launch_bounds__(1024) void setup_kernel(SetupArgs A) {
  __shared__ double sh[64];
  const int m = A.m, n = A.n, tid = threadIdx.x, nt = blockDim.x;
  double bb = 0.0, aa = 0.0, bw1 = 0.0, bw2 = 0.0;
  int bad = 0;
  for (int j = tid; j < n; j += nt) {
    const double bj = A.b[j];
    bb += bj * bj;
    bw1 += bj * A.w1[j];
    bw2 += bj * A.w2[j];
    if (!isfinite(bj)) bad |= kStNonFinite;
  }
  for (int j = tid; j < m; j += nt) {
    const double aj = A.a[j], sj = A.sigma[j];
    aa += aj * aj;
    if (!isfinite(aj) || !isfinite(sj)) bad |= kStNonFinite;
    if (sj < 0.0 || (j > 0 && A.sigma[j - 1] < sj)) bad |= kStBadSigma;
  }
  bb = block_sum(bb, sh);
  aa = block_sum(aa, sh);
  bw1 = block_sum(bw1, sh);
  bw2 = block_sum(bw2, sh);
  if (bad) atomicOr(A.status, bad);
  double r1, r2, r3, r4, Qu[4], Qv[4];
  gram_split_dev(bb, &r1, &r2, Qu);
  gram_split_dev(aa, &r3, &r4, Qv);
  if (tid == 0) {
    A.scal[0] = bb;
    A.scal[1] = aa;
    A.scal[2] = bw1;
    A.scal[3] = bw2;
    *A.rho1 = r1;
    *A.rho2 = r2;
    *A.rho3 = r3;
    *A.rho4 = r4;
  }
  for (int j = tid; j < m; j += nt) {
    const double sj = A.sigma[j];
    const double pj = A.p[j], sq = sj * A.q[j];
    A.zLp[j] = Qu[0] * pj + Qu[2] * sq;   // U^T a1
    A.yLm[j] = Qu[1] * pj + Qu[3] * sq;   // U^T b1
    A.pL1[j] = sj * A.t1[j] + pj * bw1;   // U^T A^ w1
    A.pL2[j] = sj * A.t2[j] + pj * bw2;
    A.lamLp[j] = sj * sj;
    A.colLp[j] = m - 1 - j;               // ascending position -> column (sigma descending)
    A.colLm[j] = j;
  }
  for (int j = tid; j < n; j += nt) {
    const double sp = (j < m) ? A.sigma[j] * A.p[j] : 0.0;  // S^T p
    const double qj = A.q[j];
    A.zRp[j] = Qv[0] * qj + Qv[2] * sp;   // V^T a2
    A.yRm[j] = Qv[1] * qj + Qv[3] * sp;   // V^T b2
    A.lamRp[j] = (j < m) ? A.sigma[j] * A.sigma[j] : 0.0;
    A.colRp[j] = (j < n - m) ? m + j : m - 1 - (j - (n - m));
    A.colRm[j] = j;
  }
}

__global__ void finalize_kernel(int m, int n, const double* lamL, const double* fL1, const double* fL2,
                                const double* fR1, const double* fR2, double* sigma_out, double* signs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    sigma_out[i] = sqrt(fmax(lamL[i], 0.0));
    const double p1 = fL1[i] * fR1[i], p2 = fL2[i] * fR2[i];
    const double p = (fabs(p1) >= fabs(p2)) ? p1 : p2;
    signs[i] = (p < 0.0) ? -1.0 : 1.0;
  } else if (i < n) {
    signs[i] = 1.0;
  }
}

__global__ void nonfinite_check(int R, int N, const double* X, int ldx, int* status) {
  // one pass over a factor; a thread per column, rows strided by the grid
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  bool bad = false;
  for (int r = blockIdx.y; r < R; r += gridDim.y) bad |= !isfinite(X[(size_t)r * ldx + j]);
  if (bad) atomicOr(status, (int)kStNonFinite);
}

// Copies N flags and zero-fills the row up to `width`.
__global__ void copy_flags(int N, int width, const int8_t* src, int8_t* dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < width) dst[j] = (j < N) ? src[j] : 0;
}

__global__ void set_scalar(double* dst, double v, int* status) {
  if (threadIdx.x == 0) {
    *dst = v;
    if (status) status[0] = 0;
  }
}

__global__ void identity_map(int N, int* col) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) col[j] = j;
}

__global__ void square_kernel(int N, const double* z, double* w2, int* Kdev, int K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *Kdev = K;
  if (j < N) w2[j] = z[j] * z[j];
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

int hip_ok() { return hipGetLastError() == hipSuccess ? SVDU_OK : SVDU_EHIP; }

// Host copies of one stage's roots, for the FMM plans.
struct HostRoots {
  int counts[4];
  std::vector<double> g, tau;
  std::vector<int> org;
};

void enqueue_root_copies(const Stage& s, HostRoots* h, hipStream_t st) {
  h->g.resize(s.N);
  h->tau.resize(s.N);
  h->org.resize(s.N);
  (void)hipMemcpyAsync(h->counts, s.counts, sizeof(h->counts), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h->g.data(), s.g, s.N * sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h->tau.data(), s.tau, s.N * sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h->org.data(), s.org, s.N * sizeof(int), hipMemcpyDeviceToHost, st);
}

// The four products through the FMM. One host round trip: the roots of all
// four eigen-updates come to the host, the tree plans are built and uploaded
// in one copy, then the kernels are enqueued.
int fmm_products_impl(int nst, Stage* stages, const int* Rs, const double* const* Xs, const int* ldxs,
                      double* const* Xos, const int* ldos, const double* const* scales, const int* status_dev,
                      double* work, size_t work_elems, char* plan_dev, size_t plan_bytes, double eps,
                      std::vector<int> marks, int tcall, hipStream_t st) {
  std::vector<HostRoots> h(nst);
  int status = 0;
  (void)hipMemcpyAsync(&status, status_dev, sizeof(int), hipMemcpyDeviceToHost, st);
  for (int k = 0; k < nst; ++k) enqueue_root_copies(stages[k], &h[k], st);
  if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;
  if (status & kStFatal) return SVDU_OK;   // reported by svdu_get_status
  std::vector<char> blob;
  std::vector<FmmPrepared> prep(nst);
  for (int k = 0; k < nst; ++k) {
    const int K = h[k].counts[0];
    std::vector<double> mu(K);
    for (int i = 0; i < K; ++i) mu[i] = h[k].g[h[k].org[i]] + h[k].tau[i];
    fmm_prepare(K, h[k].g.data(), mu.data(), eps, &blob, &prep[k]);
  }
  if (blob.size() > plan_bytes) return SVDU_ENOMEM;
  if (!blob.empty()) {
    if (hipMemcpyAsync(plan_dev, blob.data(), blob.size(), hipMemcpyHostToDevice, st) != hipSuccess) return SVDU_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;   // blob is a host temporary
  }
  for (int k = 0; k < nst; ++k) {
    if (fmm_launch(Rs[k], Xs[k], ldxs[k], stages[k], prep[k], plan_dev, Xos[k], ldos[k], scales[k], work,
                   work_elems, st) != 0)
      return SVDU_ENOMEM;
    if (k < (int)marks.size()) ring_mark(tcall, marks[k], st);
  }
  return SVDU_OK;
}

int fmm_products(Layout& L, int m, int n, const double* U, int ldu, const double* V, int ldv, double* U_out,
                 int ldu_out, double* V_out, int ldv_out, double eps, int tcall, hipStream_t st) {
  // the two sides share the intermediate T, so they run one after the other
  {
    Stage st2[2] = {L.st[0], L.st[1]};
    const int Rs[2] = {m, m};
    const double* Xs[2] = {U, L.T};
    const int ldx[2] = {ldu, m};
    double* Xo[2] = {L.T, U_out};
    const int ldo[2] = {m, ldu_out};
    const double* sc[2] = {nullptr, nullptr};
    const int rc = fmm_products_impl(2, st2, Rs, Xs, ldx, Xo, ldo, sc, L.status, L.fmm_work, L.fmm_elems,
                                     L.fmm_plan, L.fmm_plan_bytes, eps, {3, 4}, tcall, st);
    if (rc != SVDU_OK) return rc;
  }
  {
    Stage st2[2] = {L.st[2], L.st[3]};
    const int Rs[2] = {n, n};
    const double* Xs[2] = {V, L.T};
    const int ldx[2] = {ldv, n};
    double* Xo[2] = {L.T, V_out};
    const int ldo[2] = {n, ldv_out};
    const double* sc[2] = {nullptr, L.signs};
    return fmm_products_impl(2, st2, Rs, Xs, ldx, Xo, ldo, sc, L.status, L.fmm_work, L.fmm_elems, L.fmm_plan,
                             L.fmm_plan_bytes, eps, {5, 6}, tcall, st);
  }
}

}  // namespace
}  // namespace svdu

using namespace svdu;

extern "C" {

size_t svdu_workspace_bytes(int m, int n, int path, int precision) {
  (void)path;
  (void)precision;
  if (m < 1 || n < m) return 0;
  return carve_update(nullptr, m, n, path).bytes;
}

int svdu_rank1_update(int m, int n, const double* U, int ldu, const double* sigma, const double* V, int ldv,
                      const double* a, const double* b, double eps, int path, int precision, double* U_out,
                      int ldu_out, double* sigma_out, double* V_out, int ldv_out, int8_t* defl,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (m < 1 || n < m) return SVDU_EINVAL;
  if (!U || !sigma || !V || !a || !b || !U_out || !sigma_out || !V_out || !workspace) return SVDU_EINVAL;
  if (ldu < m || ldv < n || ldu_out < m || ldv_out < n) return SVDU_EINVAL;
  if (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM) return SVDU_EINVAL;
  if (precision != SVDU_PREC_FP64 && precision != SVDU_PREC_SPLIT32) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && !(eps > 0.0 && eps < 1.0)) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && precision != SVDU_PREC_FP64) return SVDU_ENOTSUP;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  const size_t ub = ((size_t)(m - 1) * ldu + m) * 8, vb = ((size_t)(n - 1) * ldv + n) * 8;
  const size_t uob = ((size_t)(m - 1) * ldu_out + m) * 8, vob = ((size_t)(n - 1) * ldv_out + n) * 8;
  if (overlaps(U, ub, U_out, uob) || overlaps(V, vb, V_out, vob) || overlaps(U_out, uob, V_out, vob))
    return SVDU_EINVAL;
  Layout L = carve_update(workspace, m, n, path);
  if (workspace_bytes < L.bytes) return SVDU_ENOMEM;
  if (overlaps(workspace, L.bytes, U_out, uob) || overlaps(workspace, L.bytes, V_out, vob)) return SVDU_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int tcall = ring_begin();
  ring_mark(tcall, 0, st);

  // 1. status word and probes
  hipLaunchKernelGGL(init_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, L.status, L.w1, L.w2);
  {
    const int gy = std::min(64, std::max(1, n / 64));
    hipLaunchKernelGGL(nonfinite_check, dim3((m + 255) / 256, std::min(gy, m)), dim3(256), 0, st, m, m, U, ldu,
                       L.status);
    hipLaunchKernelGGL(nonfinite_check, dim3((n + 255) / 256, gy), dim3(256), 0, st, n, n, V, ldv, L.status);
  }
  // 2. projections
  launch_gemv_t(m, m, U, ldu, 1, a, nullptr, nullptr, L.p, nullptr, nullptr, L.gemv_scratch, L.gemv_elems, st);
  launch_gemv_t(n, n, V, ldv, 3, b, L.w1, L.w2, L.q, L.t1, L.t2, L.gemv_scratch, L.gemv_elems, st);
  ring_mark(tcall, 1, st);
  // 3. splits and core-space vectors
  Stage& sLp = L.st[0];
  Stage& sLm = L.st[1];
  Stage& sRp = L.st[2];
  Stage& sRm = L.st[3];
  SetupArgs A{m,         n,        sigma,    a,        b,        L.p,      L.q,      L.t1,     L.t2,
              L.w1,      L.w2,     L.scal,   L.status, sLp.rho,  sLm.rho,  sRp.rho,  sRm.rho,  L.zLp,
              L.yLm,     L.pL1,    L.pL2,    L.lamLp,  L.zRp,    L.yRm,    L.lamRp,  sLp.col_of,
              sLm.col_of, sRp.col_of, sRm.col_of};
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(1024), 0, st, A);
  // 4. eigen-updates
  for (int k = 0; k < 4; ++k) L.st[k].status = L.status;
  sLp.N = m; sLp.lam_in = L.lamLp; sLp.z = L.zLp; sLp.descending = false;
  sLm.N = m; sLm.lam_in = sLp.lam_out; sLm.z = L.zLm; sLm.descending = true;
  sRp.N = n; sRp.lam_in = L.lamRp; sRp.z = L.zRp; sRp.descending = false;
  sRm.N = n; sRm.lam_in = sRp.lam_out; sRm.z = L.zRm; sRm.descending = true;
  {
    launch_stage_small(sLp, g_maxit, st);
    const double* x[3] = {L.yLm, L.pL1, L.pL2};
    double* y[3] = {L.zLm, L.pL1b, L.pL2b};
    launch_cauchy_tmatvec(sLp, 3, x, y, st);
    launch_stage_small(sLm, g_maxit, st);
    const double* x2[2] = {L.pL1b, L.pL2b};
    double* y2[2] = {L.fL1, L.fL2};
    launch_cauchy_tmatvec(sLm, 2, x2, y2, st);
  }
  {
    launch_stage_small(sRp, g_maxit, st);
    const double* x[3] = {L.yRm, L.t1, L.t2};
    double* y[3] = {L.zRm, L.pR1b, L.pR2b};
    launch_cauchy_tmatvec(sRp, 3, x, y, st);
    launch_stage_small(sRm, g_maxit, st);
    const double* x2[2] = {L.pR1b, L.pR2b};
    double* y2[2] = {L.fR1, L.fR2};
    launch_cauchy_tmatvec(sRm, 2, x2, y2, st);
  }
  // 5. singular values and signs
  hipLaunchKernelGGL(finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, st, m, n, sLm.lam_out, L.fL1, L.fL2,
                     L.fR1, L.fR2, sigma_out, L.signs);
  ring_mark(tcall, 2, st);
  // 6. products: FP64 MFMA (direct), split-FP32 MFMA plus an FP64 column
  //    renormalisation (precision form), or the row-batched FMM
  if (path == SVDU_PATH_FMM) {
    const int rc = fmm_products(L, m, n, U, ldu, V, ldv, U_out, ldu_out, V_out, ldv_out, eps, tcall, st);
    if (rc != SVDU_OK) return rc;
  } else {
    auto product = [&](int R, const double* X, int ldx, const CauchyDesc& d, double* Xo, int ldo) {
      if (precision == SVDU_PREC_SPLIT32)
        launch_gemm_cauchy_split32(R, X, ldx, d, Xo, ldo, st);
      else
        launch_gemm_cauchy_f64(R, X, ldx, d, Xo, ldo, st);
    };
    product(m, U, ldu, desc_of(sLp), L.T, m);
    ring_mark(tcall, 3, st);
    product(m, L.T, m, desc_of(sLm), U_out, ldu_out);
    ring_mark(tcall, 4, st);
    product(n, V, ldv, desc_of(sRp), L.T, n);
    ring_mark(tcall, 5, st);
    product(n, L.T, n, desc_of(sRm, L.signs), V_out, ldv_out);
    if (precision == SVDU_PREC_SPLIT32) {
      launch_column_renorm(m, m, U_out, ldu_out, L.renorm_scratch, L.status, st);
      launch_column_renorm(n, n, V_out, ldv_out, L.renorm_scratch, L.status, st);
    }
  }
  ring_mark(tcall, 6, st);
  if (defl) {
    for (int k = 0; k < 4; ++k) {
      hipLaunchKernelGGL(copy_flags, dim3((n + 255) / 256), dim3(256), 0, st, L.st[k].N, n, L.st[k].flags,
                         defl + (size_t)k * n);
    }
  }
  ring_mark(tcall, 7, st);
  return hip_ok();
}

int svdu_timing_read(double* ms, int max_calls) {
  const int n = std::min(g_ring.count, max_calls);
  for (int c = 0; c < n; ++c) {
    if (hipEventSynchronize(g_ring.ev[c][kRingEvents - 1]) != hipSuccess) return SVDU_EHIP;
    for (int k = 0; k + 1 < kRingEvents; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, g_ring.ev[c][k], g_ring.ev[c][k + 1]) != hipSuccess) return SVDU_EHIP;
      ms[c * (kRingEvents - 1) + k] = t;
    }
  }
  return n;
}

int svdu_get_status(const void* workspace, void* stream) {
  if (!workspace) return SVDU_EINVAL;
  int h = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(&h, workspace, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return SVDU_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;
  if (h & kStNonFinite) return SVDU_ENONFINITE;
  if (h & kStBadSigma) return SVDU_EBADSIGMA;
  if (h & kStNoConv) return SVDU_ENOCONV;
  return SVDU_OK;
}

struct EigLayout {
  Stage st;
  int* status;
  double* fmm_work;
  size_t fmm_elems;
  char* fmm_plan;
  size_t fmm_plan_bytes;
  size_t bytes;
};

static EigLayout carve_eig(void* ws, int R, int N, int path) {
  Carver c(ws);
  EigLayout E;
  E.status = c.take<int>(16);
  carve_stage(c, E.st, N);
  E.st.N = N;
  E.fmm_elems = (path == SVDU_PATH_FMM) ? fmm_workspace_elems(std::max(R, 1), N) : 0;
  E.fmm_work = c.take<double>(E.fmm_elems);
  E.fmm_plan_bytes = (path == SVDU_PATH_FMM) ? fmm_plan_bytes(N) : 0;
  E.fmm_plan = c.take<char>(E.fmm_plan_bytes);
  E.bytes = c.off + 256;
  return E;
}

size_t svdu_eig_update_workspace_bytes(int R, int N, int path) {
  if (N < 1 || R < 0 || (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM)) return 0;
  return carve_eig(nullptr, R, N, path).bytes;
}

int svdu_eig_update(int R, int N, const double* X, int ldx, const double* lam, const double* z, double rho, int path,
                    double eps, double* X_out, int ldo, double* lam_out, int8_t* defl, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (R < 0 || N < 1 || ldx < N || ldo < N || !lam || !z || !workspace || !lam_out) return SVDU_EINVAL;
  if (R > 0 && (!X || !X_out)) return SVDU_EINVAL;
  if (!(rho != 0.0) || !isfinite(rho)) return SVDU_EINVAL;
  if (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && !(eps > 0.0 && eps < 1.0)) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  if (R > 0 && overlaps(X, ((size_t)(R - 1) * ldx + N) * 8, X_out, ((size_t)(R - 1) * ldo + N) * 8))
    return SVDU_EINVAL;
  EigLayout E = carve_eig(workspace, R, N, path);
  if (workspace_bytes < E.bytes) return SVDU_ENOMEM;
  Stage& s = E.st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(set_scalar, dim3(1), dim3(64), 0, st, s.rho, rho, E.status);
  hipLaunchKernelGGL(identity_map, dim3((N + 255) / 256), dim3(256), 0, st, N, s.col_of);
  s.lam_in = lam;
  s.z = const_cast<double*>(z);
  s.descending = false;
  s.status = E.status;
  launch_stage_small(s, g_maxit, st);
  if (path == SVDU_PATH_FMM) {
    const int Rs[1] = {R};
    const double* Xs[1] = {X};
    const int ldxs[1] = {ldx};
    double* Xos[1] = {X_out};
    const int ldos[1] = {ldo};
    const double* sc[1] = {nullptr};
    const int rc = fmm_products_impl(1, &s, Rs, Xs, ldxs, Xos, ldos, sc, E.status, E.fmm_work, E.fmm_elems,
                                     E.fmm_plan, E.fmm_plan_bytes, eps, {}, -1, st);
    if (rc != SVDU_OK) return rc;
  } else {
    launch_gemm_cauchy_f64(R, X, ldx, desc_of(s), X_out, ldo, st);
  }
  if (hipMemcpyAsync(lam_out, s.lam_out, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return SVDU_EHIP;
  if (defl) hipLaunchKernelGGL(copy_flags, dim3((N + 255) / 256), dim3(256), 0, st, N, N, s.flags, defl);
  return hip_ok();
}

size_t svdu_secular_workspace_bytes(int K) {
  if (K < 1) return 0;
  Carver c(nullptr);
  c.take<int>(16);
  c.take<int>(4);
  c.take<double>(1);
  c.take<double>(K);
  return c.off + 256;
}

int svdu_secular(int K, const double* d, const double* z, double rho, int* org, double* tau, int* iters,
                 void* workspace, size_t workspace_bytes, void* stream) {
  if (K < 1 || !d || !z || !org || !tau || !workspace) return SVDU_EINVAL;
  if (!(rho != 0.0) || !isfinite(rho)) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  if (workspace_bytes < svdu_secular_workspace_bytes(K)) return SVDU_ENOMEM;
  Carver c(workspace);
  int* status = c.take<int>(16);
  int* Kdev = c.take<int>(4);
  double* rhod = c.take<double>(1);
  double* w2 = c.take<double>(K);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(set_scalar, dim3(1), dim3(64), 0, st, rhod, rho, status);
  hipLaunchKernelGGL(square_kernel, dim3((K + 255) / 256), dim3(256), 0, st, K, z, w2, Kdev, K);
  launch_secular(K, Kdev, d, w2, rhod, org, tau, iters, status, g_maxit, st);
  return hip_ok();
}

int svdu_set_option(int option, int value) {
  if (option == SVDU_OPT_SECULAR_MAXIT) {
    const int old = g_maxit;
    g_maxit = value < 1 ? 1 : value;
    return old;
  }
  if (option == SVDU_OPT_GEMM_VARIANT) {
    if (value < 1 || value > 2) return SVDU_EINVAL;
    return set_gemm_variant(value);
  }
  if (option == SVDU_OPT_TIMING) {
    const int old = g_ring.on ? 1 : 0;
    g_ring.on = value != 0;
    g_ring.count = 0;
    return old;
  }
  return SVDU_EINVAL;
}

const char* svdu_status_string(int status) {
  switch (status) {
    case SVDU_OK: return "ok";
    case SVDU_EINVAL: return "invalid argument";
    case SVDU_ENOMEM: return "workspace too small";
    case SVDU_EHIP: return "HIP runtime error";
    case SVDU_ENONFINITE: return "non-finite input";
    case SVDU_EBADSIGMA: return "sigma not descending or negative";
    case SVDU_ENOCONV: return "secular iteration cap reached";
    case SVDU_ENOTSUP: return "path/precision not available";
    default: return "unknown status";
  }
}

}  // extern "C"
