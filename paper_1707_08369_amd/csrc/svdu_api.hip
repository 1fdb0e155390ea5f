// C ABI of libsvdu for single problems: argument checks, the workspace
// layout, and the launch sequence of one rank-1 SVD update (Section 6.1 of
// the paper), one symmetric rank-one eigen-update (Section 6.2) or one secular
// solve. The sequence itself is in engine.hip; the batched entry points are
// in svdu_batch.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/svdu.h"
#include "device_util.h"
#include "engine.h"
#include "fmm_plan.h"
#include "svdu_internal.h"

namespace svdu {

// A context is required by every call that enqueues work, and the call must
// run with the context's device current (checked after the host-side argument
// checks, right before the first HIP call).
int ctx_device_check(const svdu_ctx* ctx) {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess) return SVDU_EHIP;
  return d == ctx->device ? SVDU_OK : SVDU_EINVAL;
}

namespace {

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

// acc = bits (first) or acc |= bits: the status words of a sequence of updates.
__global__ void or_status(int* acc, const int* bits, int first) {
  if (threadIdx.x == 0) *acc = first ? *bits : (*acc | *bits);
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

// Host copies of one stage's roots, for the FMM plans: views into host
// memory that the caller owns.
struct HostRoots {
  int* counts;   // 4
  double* g;     // N
  double* tau;   // N
  int* org;      // N
};

// Host memory for the roots of one stage of order N: counts, g, tau, org.
static size_t host_roots_bytes(int N) { return ((size_t)16 + 20 * (size_t)N + 255) & ~size_t(255); }

static HostRoots host_roots_at(char* p, int N) {
  HostRoots h;
  h.counts = reinterpret_cast<int*>(p);
  h.g = reinterpret_cast<double*>(p + 16);
  h.tau = h.g + N;
  h.org = reinterpret_cast<int*>(h.tau + N);
  return h;
}

void enqueue_root_copies(const Stage& s, const HostRoots& h, hipStream_t st) {
  (void)hipMemcpyAsync(h.counts, s.counts, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h.g, s.g, s.N * sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h.tau, s.tau, s.N * sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(h.org, s.org, s.N * sizeof(int), hipMemcpyDeviceToHost, st);
}

// The tree plan of one product from the host copies of its stage's roots
// (appended to blob). The host reads indices that the device produced: they
// are checked before use, so inconsistent device results give an error
// instead of a host fault.
int prepare_plan(const Stage& s, const HostRoots& h, double eps, std::vector<char>* blob, FmmPrepared* pp) {
  const int K = h.counts[0];
  if (K < 0 || K > s.N) return SVDU_EHIP;
  std::vector<double> mu(K);
  for (int i = 0; i < K; ++i) {
    const int o = h.org[i];
    if (o < 0 || o >= K) return SVDU_EHIP;
    mu[i] = h.g[o] + h.tau[i];
  }
  fmm_prepare(K, h.g, mu.data(), eps, blob, pp);
  return SVDU_OK;
}

// Products through the FMM for a list of eigen-updates. One host round
// trip: their roots come to the host, the tree plans are built and uploaded in
// one copy, then the kernels are enqueued.
int fmm_products_impl(int nst, Stage* stages, const int* Rs, const double* const* Xs, const int* ldxs,
                      double* const* Xos, const int* ldos, const double* const* scales, const int* status_dev,
                      double* work, size_t work_elems, char* plan_dev, size_t plan_bytes, double eps,
                      hipStream_t st) {
  std::vector<size_t> at(nst + 1, 0);
  for (int k = 0; k < nst; ++k) at[k + 1] = at[k] + host_roots_bytes(stages[k].N);
  std::vector<double> mem((at[nst] + 7) / 8);   // 8-byte aligned; the call waits for its copies below
  std::vector<HostRoots> h(nst);
  int status = 0;
  (void)hipMemcpyAsync(&status, status_dev, sizeof(int), hipMemcpyDeviceToHost, st);
  for (int k = 0; k < nst; ++k) {
    h[k] = host_roots_at(reinterpret_cast<char*>(mem.data()) + at[k], stages[k].N);
    enqueue_root_copies(stages[k], h[k], st);
  }
  if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;
  if (status & kStFatal) return SVDU_OK;   // reported by svdu_get_status
  std::vector<char> blob;
  std::vector<FmmPrepared> prep(nst);
  for (int k = 0; k < nst; ++k)
    if (const int rc = prepare_plan(stages[k], h[k], eps, &blob, &prep[k])) return rc;
  if (blob.size() > plan_bytes) return SVDU_ENOMEM;
  if (!blob.empty()) {
    if (hipMemcpyAsync(plan_dev, blob.data(), blob.size(), hipMemcpyHostToDevice, st) != hipSuccess) return SVDU_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;   // blob is a host temporary
  }
  for (int k = 0; k < nst; ++k)
    if (fmm_launch(Rs[k], Xs[k], ldxs[k], stages[k], prep[k], plan_dev, Xos[k], ldos[k], scales[k], work,
                   work_elems, st) != 0)
      return SVDU_ENOMEM;
  return SVDU_OK;
}

// The context's other streams and the events of the FMM path (made on first
// use, on the context's device, which is current).
static bool fmm_sync_objects(svdu_ctx* ctx) {
  auto event = [](hipEvent_t* e) {
    if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) *e = nullptr;
    return *e != nullptr;
  };
  auto stream = [](hipStream_t* s) {
    if (!*s && hipStreamCreateWithFlags(s, hipStreamNonBlocking) != hipSuccess) *s = nullptr;
    return *s != nullptr;
  };
  const bool ss = stream(&ctx->aux) && stream(&ctx->aux2);
  const bool ev = event(&ctx->fork) && event(&ctx->join) && event(&ctx->roots[0]) && event(&ctx->roots[1]) &&
                  event(&ctx->up0) && event(&ctx->done_a) && event(&ctx->done_b) && event(&ctx->uploaded);
  return ss && ev;
}

// The whole update on the FMM path, from the projections to the products
// (the caller enqueues the rest). The products run by level: U C~_L+ -> TL
// and V C~_R+ -> TR, then TL C~_L- -> U^ and TR C~_R- diag(s) -> V^. The tree
// plans are built on the host from the roots, so each level's roots are
// copied into pinned host memory as soon as its eigen-updates are enqueued:
//  * level 0: once its roots arrive, the host builds its plans while the
//    device runs the level-1 eigen-updates; the plans are uploaded and the
//    two products run on the context's two other streams, beside those
//    eigen-updates (they only read U, V and the level-0 descriptors);
//  * level 1: the host builds its plans while the level-0 products run; the
//    caller's stream uploads them, waits for the level-0 products, and runs
//    the left-hand product while the second stream runs the right-hand one.
// Every stream is joined back into the caller's stream before the call
// returns, also after an error. Results do not depend on the overlap.
int fmm_update(svdu_ctx* ctx, const Update& u, const Plan& P, double eps, const Sched& S, hipStream_t st) {
  const Layout& L = u.L;
  if (!fmm_sync_objects(ctx)) return SVDU_EHIP;
  if (ctx->upload_pending) {   // the last call's uploads read the pinned memory
    if (hipEventSynchronize(ctx->uploaded) != hipSuccess) return SVDU_EHIP;
    ctx->upload_pending = false;
  }
  struct LevelHost {
    HostRoots h[2];   // the left and the right eigen-update of the level
    int* status;
    hipEvent_t ev;
    char* blob;       // pinned staging of the level's plans
  } H[2];
  // pinned host memory: 256 bytes of status words, the roots, then one plan
  // staging area per level
  const size_t half = (L.fmm_plan_bytes / 2) & ~size_t(255);   // the plans of one level (two products)
  size_t need = 256;
  for (int k = 0; k < 4; ++k) need += host_roots_bytes(P.host_stages[k].N);
  need += 2 * half;
  if (need > ctx->pinned_bytes) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    if (hipHostMalloc(&ctx->pinned, need, hipHostMallocDefault) != hipSuccess) {
      ctx->pinned = nullptr;
      return SVDU_EHIP;
    }
    ctx->pinned_bytes = need;
  }
  {
    char* p = static_cast<char*>(ctx->pinned);
    H[0].ev = ctx->roots[0];
    H[1].ev = ctx->roots[1];
    H[0].status = reinterpret_cast<int*>(p);
    H[1].status = H[0].status + 1;
    size_t at = 256;
    for (int lev = 0; lev < 2; ++lev)
      for (int side = 0; side < 2; ++side) {
        const int N = P.host_stages[2 * side + lev].N;
        H[lev].h[side] = host_roots_at(p + at, N);
        at += host_roots_bytes(N);
      }
    H[0].blob = p + at;
    H[1].blob = p + at + half;
  }
  const std::function<void(int)> copy_roots = [&](int lev) {
    (void)hipMemcpyAsync(H[lev].status, L.status, sizeof(int), hipMemcpyDeviceToHost, st);
    for (int side = 0; side < 2; ++side) enqueue_root_copies(P.host_stages[2 * side + lev], H[lev].h[side], st);
    (void)hipEventRecord(H[lev].ev, st);
  };
  enqueue_plan(P, S, kStepUpToRoots, st, &copy_roots);
  // one product of level lev, side 0 (left) or 1 (right)
  auto product = [&](int lev, int side, const FmmPrepared& pp, const char* plan, hipStream_t s) {
    const bool left = side == 0;
    const int N = left ? u.m : u.n;
    const double* X = lev == 0 ? (left ? u.U : u.V) : (left ? L.TL : L.TR);
    const int ldx = lev == 0 ? (left ? u.ldu : u.ldv) : N;
    double* Xo = lev == 0 ? (left ? L.TL : L.TR) : (left ? u.U_out : u.V_out);
    const int ldo = lev == 0 ? N : (left ? u.ldu_out : u.ldv_out);
    const double* sc = (lev == 1 && !left) ? L.signs : nullptr;
    return fmm_launch(N, X, ldx, P.host_stages[2 * side + lev], pp, plan, Xo, ldo, sc,
                      left ? L.fmm_work_l : L.fmm_work, left ? L.fmm_elems_l : L.fmm_elems, s) == 0
               ? SVDU_OK
               : SVDU_ENOMEM;
  };
  // the plans of level lev from its roots, staged in pinned memory; size in *bytes
  auto plans = [&](int lev, FmmPrepared (&prep)[2], size_t* bytes) {
    std::vector<char> blob;
    for (int side = 0; side < 2; ++side)
      if (const int rc = prepare_plan(P.host_stages[2 * side + lev], H[lev].h[side], eps, &blob, &prep[side]))
        return rc;
    if (blob.size() > half) return SVDU_ENOMEM;
    if (!blob.empty()) memcpy(H[lev].blob, blob.data(), blob.size());
    *bytes = blob.size();
    return SVDU_OK;
  };
  int rc = SVDU_OK;
  bool level0 = false;   // level-0 work was enqueued on the other streams
  do {
    // level 0, on the two other streams
    if (hipEventSynchronize(H[0].ev) != hipSuccess) {
      rc = SVDU_EHIP;
      break;
    }
    if (*H[0].status & kStFatal) break;   // reported by svdu_get_status
    FmmPrepared prep0[2];
    size_t bytes0 = 0;
    if ((rc = plans(0, prep0, &bytes0)) != SVDU_OK) break;
    level0 = true;
    if (hipStreamWaitEvent(ctx->aux, H[0].ev, 0) != hipSuccess ||
        (bytes0 && hipMemcpyAsync(L.fmm_plan, H[0].blob, bytes0, hipMemcpyHostToDevice, ctx->aux) != hipSuccess) ||
        hipEventRecord(ctx->up0, ctx->aux) != hipSuccess || hipStreamWaitEvent(ctx->aux2, ctx->up0, 0) != hipSuccess) {
      rc = SVDU_EHIP;
      break;
    }
    if ((rc = product(0, 0, prep0[0], L.fmm_plan, ctx->aux)) != SVDU_OK) break;
    if ((rc = product(0, 1, prep0[1], L.fmm_plan, ctx->aux2)) != SVDU_OK) break;
    // level 1, forked from the caller's stream
    if (hipEventSynchronize(H[1].ev) != hipSuccess) {
      rc = SVDU_EHIP;
      break;
    }
    if (*H[1].status & kStFatal) break;
    FmmPrepared prep1[2];
    size_t bytes1 = 0;
    if ((rc = plans(1, prep1, &bytes1)) != SVDU_OK) break;
    char* plan1 = L.fmm_plan + half;
    if (bytes1 && hipMemcpyAsync(plan1, H[1].blob, bytes1, hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = SVDU_EHIP;
      break;
    }
    if (hipEventRecord(ctx->done_a, ctx->aux) != hipSuccess || hipEventRecord(ctx->done_b, ctx->aux2) != hipSuccess ||
        hipStreamWaitEvent(st, ctx->done_a, 0) != hipSuccess || hipStreamWaitEvent(st, ctx->done_b, 0) != hipSuccess) {
      rc = SVDU_EHIP;
      break;
    }
    level0 = false;   // joined
    S.mark(3, st);
    if (hipEventRecord(ctx->fork, st) != hipSuccess || hipStreamWaitEvent(ctx->aux, ctx->fork, 0) != hipSuccess) {
      rc = SVDU_EHIP;
      break;
    }
    rc = product(1, 0, prep1[0], plan1, st);
    if (rc == SVDU_OK) rc = product(1, 1, prep1[1], plan1, ctx->aux);
    if (hipEventRecord(ctx->join, ctx->aux) != hipSuccess || hipStreamWaitEvent(st, ctx->join, 0) != hipSuccess)
      rc = SVDU_EHIP;
    if (rc == SVDU_OK) S.mark(4, st);
  } while (false);
  if (level0) {   // an exit between the levels: join the other streams all the same
    (void)hipEventRecord(ctx->done_a, ctx->aux);
    (void)hipEventRecord(ctx->done_b, ctx->aux2);
    (void)hipStreamWaitEvent(st, ctx->done_a, 0);
    (void)hipStreamWaitEvent(st, ctx->done_b, 0);
  }
  // every upload has been enqueued before this point on a stream the caller's now waits for
  if (hipEventRecord(ctx->uploaded, st) == hipSuccess) ctx->upload_pending = true;
  // the root copies write the pinned buffer: let every one finish before the call returns
  for (LevelHost& x : H) (void)hipEventSynchronize(x.ev);
  return rc;
}

// Single-update workspace: the update's layout, then 2 kNumShapes tile
// counters and its job tables.
struct SingleWs {
  Layout L;
  int* counters;
  char* tables;
  size_t bytes;
};

SingleWs carve_single(void* ws, int m, int n, int path, int precision) {
  SingleWs S;
  S.L = carve_update(ws, m, n, path, precision);
  Carver c(ws);
  c.off = S.L.bytes;
  S.counters = c.take<int>(2 * kNumShapes);
  S.tables = c.take<char>(kSingleTableBytes);
  S.bytes = c.off + 256;
  return S;
}

}  // namespace
}  // namespace svdu

using namespace svdu;

extern "C" {

size_t svdu_workspace_bytes(int m, int n, int path, int precision) {
  if (m < 1 || n < m) return 0;
  if (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM) return 0;
  if (!precision_ok(precision)) return 0;
  return carve_single(nullptr, m, n, path, precision).bytes;
}

int svdu_create(svdu_ctx** ctx, int device) {
  if (!ctx) return SVDU_EINVAL;
  *ctx = nullptr;
  if (device < 0) return SVDU_EINVAL;
  svdu_ctx* c = new (std::nothrow) svdu_ctx;
  if (!c) return SVDU_ENOMEM;
  c->device = device;
  *ctx = c;
  return SVDU_OK;
}

void svdu_destroy(svdu_ctx* ctx) { delete ctx; }

int svdu_rank1_update(svdu_ctx* ctx, int m, int n, const double* U, int ldu, const double* sigma, const double* V,
                      int ldv, const double* a, const double* b, double eps, int path, int precision, double* U_out,
                      int ldu_out, double* sigma_out, double* V_out, int ldv_out, int8_t* defl,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (!ctx) return SVDU_EINVAL;
  if (m < 1 || n < m) return SVDU_EINVAL;
  if (!U || !sigma || !V || !a || !b || !U_out || !sigma_out || !V_out || !workspace) return SVDU_EINVAL;
  if (ldu < m || ldv < n || ldu_out < m || ldv_out < n) return SVDU_EINVAL;
  if (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM) return SVDU_EINVAL;
  if (!precision_ok(precision)) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && !(eps > 0.0 && eps < 1.0)) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && fmm_required_order(eps) > kFmmMaxOrder) return SVDU_ENOTSUP;
  if (path == SVDU_PATH_FMM && precision != SVDU_PREC_FP64) return SVDU_ENOTSUP;
  if (precision == SVDU_PREC_SLICED_INT8 && n > kI8MaxN) return SVDU_ENOTSUP;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  const size_t ub = ((size_t)(m - 1) * ldu + m) * 8, vb = ((size_t)(n - 1) * ldv + n) * 8;
  const size_t uob = ((size_t)(m - 1) * ldu_out + m) * 8, vob = ((size_t)(n - 1) * ldv_out + n) * 8;
  if (overlaps(U, ub, U_out, uob) || overlaps(V, vb, V_out, vob) || overlaps(U_out, uob, V_out, vob))
    return SVDU_EINVAL;
  const SingleWs W = carve_single(workspace, m, n, path, precision);
  if (workspace_bytes < W.bytes) return SVDU_ENOMEM;
  if (overlaps(workspace, W.bytes, U_out, uob) || overlaps(workspace, W.bytes, V_out, vob)) return SVDU_EINVAL;
  if (const int rc = ctx_device_check(ctx)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);

  Update u;
  u.m = m;
  u.n = n;
  u.U = U;
  u.sigma = sigma;
  u.V = V;
  u.a = a;
  u.b = b;
  u.ldu = ldu;
  u.ldv = ldv;
  u.U_out = U_out;
  u.sigma_out = sigma_out;
  u.V_out = V_out;
  u.ldu_out = ldu_out;
  u.ldv_out = ldv_out;
  u.defl = defl;
  u.L = W.L;
  std::vector<char> blob;
  Plan P;
  build_plan({u}, precision, ctx->opt, W.tables, W.counters, &blob, &P);
  if (blob.size() > kSingleTableBytes) return SVDU_ENOMEM;
  write_blob(blob, W.tables, st);
  const Sched S = sched_of(ctx, ctx->opt, ctx->opt.persistent, true);
  if (path == SVDU_PATH_FMM) {
    const int rc = fmm_update(ctx, u, P, eps, S, st);
    if (rc != SVDU_OK) return rc;
    enqueue_plan(P, S, kStepProductsOnward, st);
  } else {
    enqueue_plan(P, S, kStepAll, st);
  }
  return hip_ok();
}

// Rank-k workspace: one rank-1 update's workspace (its status word first),
// the accumulated status of the sequence, and one intermediate factor set.
struct RankkWs {
  size_t single;
  int* acc;
  double *U, *s, *V;
  size_t bytes;
};

static RankkWs carve_rankk(void* ws, int m, int n, int k, int path, int precision) {
  RankkWs W;
  W.single = svdu_workspace_bytes(m, n, path, precision);
  Carver c(ws);
  c.off = W.single;
  W.acc = c.take<int>(16);
  const size_t mm = k > 1 ? (size_t)m * m : 0, nn = k > 1 ? (size_t)n * n : 0;
  W.U = c.take<double>(mm);
  W.s = c.take<double>(k > 1 ? m : 0);
  W.V = c.take<double>(nn);
  W.bytes = c.off + 256;
  return W;
}

size_t svdu_rankk_workspace_bytes(int m, int n, int k, int path, int precision) {
  if (k < 1 || svdu_workspace_bytes(m, n, path, precision) == 0) return 0;
  return carve_rankk(nullptr, m, n, k, path, precision).bytes;
}

int svdu_rankk_update(svdu_ctx* ctx, int m, int n, int k, const double* U, int ldu, const double* sigma,
                      const double* V, int ldv, const double* A, int lda, const double* B, int ldb, double eps,
                      int path, int precision, double* U_out, int ldu_out, double* sigma_out, double* V_out,
                      int ldv_out, void* workspace, size_t workspace_bytes, void* stream) {
  if (!ctx || k < 1 || m < 1 || n < m || !A || !B || lda < m || ldb < n || !workspace) return SVDU_EINVAL;
  if (svdu_workspace_bytes(m, n, path, precision) == 0) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  const RankkWs W = carve_rankk(workspace, m, n, k, path, precision);
  if (workspace_bytes < W.bytes) return SVDU_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // update j reads the factors update j - 1 wrote; the outputs alternate
  // between the caller's buffers and the workspace's so that the last update
  // writes the caller's
  const double *Ui = U, *si = sigma, *Vi = V;
  int ldui = ldu, ldvi = ldv;
  for (int j = 0; j < k; ++j) {
    const bool to_out = ((k - 1 - j) % 2) == 0;
    double* Uo = to_out ? U_out : W.U;
    double* so = to_out ? sigma_out : W.s;
    double* Vo = to_out ? V_out : W.V;
    const int lduo = to_out ? ldu_out : m, ldvo = to_out ? ldv_out : n;
    const int rc = svdu_rank1_update(ctx, m, n, Ui, ldui, si, Vi, ldvi, A + (size_t)j * lda, B + (size_t)j * ldb,
                                     eps, path, precision, Uo, lduo, so, Vo, ldvo, nullptr, workspace, W.single,
                                     stream);
    if (rc != SVDU_OK) return rc;
    hipLaunchKernelGGL(or_status, dim3(1), dim3(64), 0, st, W.acc, static_cast<const int*>(workspace), j == 0);
    Ui = Uo;
    si = so;
    Vi = Vo;
    ldui = lduo;
    ldvi = ldvo;
  }
  // the workspace's status word reports every update of the sequence
  hipLaunchKernelGGL(or_status, dim3(1), dim3(64), 0, st, static_cast<int*>(workspace), W.acc, 1);
  return hip_ok();
}

int svdu_timing_read(svdu_ctx* ctx, double* ms, int max_calls) {
  if (!ctx || !ms || max_calls < 0) return SVDU_EINVAL;
  return ctx->ring.read(ms, max_calls);
}

int svdu_get_status(const void* workspace, void* stream) {
  if (!workspace) return SVDU_EINVAL;
  int h = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(&h, workspace, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return SVDU_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;
  return status_code(h);
}

struct EigLayout {
  Stage st;
  int* status;
  double* fmm_work;
  size_t fmm_elems;
  char* fmm_plan;
  size_t fmm_plan_bytes;
  char* tables;
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
  E.tables = c.take<char>(kSingleTableBytes);
  E.bytes = c.off + 256;
  return E;
}

size_t svdu_eig_update_workspace_bytes(int R, int N, int path) {
  if (N < 1 || R < 0 || (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM)) return 0;
  return carve_eig(nullptr, R, N, path).bytes;
}

int svdu_eig_update(svdu_ctx* ctx, int R, int N, const double* X, int ldx, const double* lam, const double* z,
                    double rho, int path, double eps, double* X_out, int ldo, double* lam_out, int8_t* defl,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!ctx) return SVDU_EINVAL;
  if (R < 0 || N < 1 || ldx < N || ldo < N || !lam || !z || !workspace || !lam_out) return SVDU_EINVAL;
  if (R > 0 && (!X || !X_out)) return SVDU_EINVAL;
  if (!(rho != 0.0) || !isfinite(rho)) return SVDU_EINVAL;
  if (path != SVDU_PATH_DIRECT && path != SVDU_PATH_FMM) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && !(eps > 0.0 && eps < 1.0)) return SVDU_EINVAL;
  if (path == SVDU_PATH_FMM && fmm_required_order(eps) > kFmmMaxOrder) return SVDU_ENOTSUP;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  if (R > 0 && overlaps(X, ((size_t)(R - 1) * ldx + N) * 8, X_out, ((size_t)(R - 1) * ldo + N) * 8))
    return SVDU_EINVAL;
  EigLayout E = carve_eig(workspace, R, N, path);
  if (workspace_bytes < E.bytes) return SVDU_ENOMEM;
  if (const int rc = ctx_device_check(ctx)) return rc;
  Stage& s = E.st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  s.lam_in = lam;
  s.z = const_cast<double*>(z);
  s.descending = false;
  s.status = E.status;
  std::vector<char> blob;
  BlobWriter B{&blob, E.tables};
  const StageLevel lev = build_level({s}, {}, B);
  GemmList G;
  int shape = 0;
  if (path == SVDU_PATH_DIRECT && R > 0) {
    const GemmJob J = make_gemm_job(R, X, ldx, with_members(desc_of(s), s), X_out, ldo, SVDU_PREC_FP64, ctx->opt);
    shape = J.shape;
    G = build_gemm_list({J}, nullptr, B);
  }
  blob.resize((blob.size() + 15) & ~size_t(15));
  if (blob.size() > kSingleTableBytes) return SVDU_ENOMEM;
  hipLaunchKernelGGL(set_scalar, dim3(1), dim3(64), 0, st, s.rho, rho, E.status);
  hipLaunchKernelGGL(identity_map, dim3((N + 255) / 256), dim3(256), 0, st, N, s.col_of);
  write_blob(blob, E.tables, st);
  launch_stage_level(lev, ctx->opt.maxit, ctx->opt.secular_ff, st);
  if (path == SVDU_PATH_FMM) {
    const int Rs[1] = {R};
    const double* Xs[1] = {X};
    const int ldxs[1] = {ldx};
    double* Xos[1] = {X_out};
    const int ldos[1] = {ldo};
    const double* sc[1] = {nullptr};
    const int rc = fmm_products_impl(1, &s, Rs, Xs, ldxs, Xos, ldos, sc, E.status, E.fmm_work, E.fmm_elems,
                                     E.fmm_plan, E.fmm_plan_bytes, eps, st);
    if (rc != SVDU_OK) return rc;
  } else {
    launch_gemm_f64(G, shape, false, 0, st);
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
  c.take<char>(kSingleTableBytes);
  return c.off + 256;
}

int svdu_secular(svdu_ctx* ctx, int K, const double* d, const double* z, double rho, int* org, double* tau,
                 int* iters, void* workspace, size_t workspace_bytes, void* stream) {
  if (!ctx) return SVDU_EINVAL;
  if (K < 1 || !d || !z || !org || !tau || !workspace) return SVDU_EINVAL;
  if (!(rho != 0.0) || !isfinite(rho)) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  if (workspace_bytes < svdu_secular_workspace_bytes(K)) return SVDU_ENOMEM;
  if (const int rc = ctx_device_check(ctx)) return rc;
  Carver c(workspace);
  int* status = c.take<int>(16);
  int* Kdev = c.take<int>(4);
  double* rhod = c.take<double>(1);
  double* w2 = c.take<double>(K);
  char* tables = c.take<char>(kSingleTableBytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // a stage whose K clusters are the K given poles
  Stage s;
  s.N = K;
  s.status = status;
  s.rho = rhod;
  s.counts = Kdev;
  s.g = const_cast<double*>(d);
  s.W2 = w2;
  s.org = org;
  s.tau = tau;
  s.iters = iters;
  std::vector<char> blob;
  BlobWriter B{&blob, tables};
  const StageLevel lev = build_level({s}, {}, B);
  blob.resize((blob.size() + 15) & ~size_t(15));
  hipLaunchKernelGGL(set_scalar, dim3(1), dim3(64), 0, st, rhod, rho, status);
  hipLaunchKernelGGL(square_kernel, dim3((K + 255) / 256), dim3(256), 0, st, K, z, w2, Kdev, K);
  write_blob(blob, tables, st);
  launch_secular_level(lev, ctx->opt.maxit, ctx->opt.secular_ff, st);
  return hip_ok();
}

int svdu_set_option(svdu_ctx* ctx, int option, int value) {
  if (!ctx) return SVDU_EINVAL;
  Options& o = ctx->opt;
  if (option == SVDU_OPT_SECULAR_MAXIT) {
    const int old = o.maxit;
    o.maxit = value < 1 ? 1 : value;
    return old;
  }
  if (option == SVDU_OPT_TILE_SHAPE) {
    if (value < -1 || value >= kNumShapes) return SVDU_EINVAL;
    const int old = o.forced_shape;
    o.forced_shape = value;
    return old;
  }
  if (option == SVDU_OPT_PERSISTENT) {
    const int old = o.persistent ? 1 : 0;
    o.persistent = value != 0;
    return old;
  }
  if (option == SVDU_OPT_REFINE) {
    const int old = o.refine ? 1 : 0;
    o.refine = value != 0;
    return old;
  }
  if (option == SVDU_OPT_SLICES) {
    if (value < kMinSlices || value > kMaxSlices) return SVDU_EINVAL;
    const int old = o.slices;
    o.slices = value;
    return old;
  }
  if (option == SVDU_OPT_SECULAR_FMM) {
    if (value < 0 || value > 2) return SVDU_EINVAL;
    const int old = o.secular_ff;
    o.secular_ff = value;
    return old;
  }
  if (option == SVDU_OPT_TIMING) return ctx->ring.set(value != 0);
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
