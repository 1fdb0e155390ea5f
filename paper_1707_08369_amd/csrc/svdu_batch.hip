// Batched rank-1 SVD updates: many independent problems of uneven sizes in
// one launch sequence (every step is one launch over all problems, see
// engine.hip), optionally captured once into a HIP graph and replayed with a
// single launch. Also the autotuner that picks the tile shape of the product
// kernels per size bucket by timing them on the device.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/svdu.h"
#include "device_util.h"
#include "engine.h"

using namespace svdu;

struct svdu_batch {
  svdu_ctx* ctx = nullptr;       // records eager launches in its timing ring
  Options opt;                   // the context's options when the batch was created
  int count = 0;
  int precision = 0;
  bool persistent = false;
  std::vector<Update> ups;
  Plan plan;
  int* status_dev = nullptr;
  int* counters = nullptr;
  char* tables = nullptr;
  char* pinned = nullptr;        // host copy of the tables (pinned), alive until destroy
  int* status_host = nullptr;    // pinned
  hipEvent_t uploaded = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int cdiv(int a, int b) { return (a + b - 1) / b; }

constexpr int kTuneTiles = 4096;                       // tuning workload per bucket, in 128 x 128 tiles
constexpr int kTuneOrders = 4;                         // orders per bucket, spread over it up to its top
constexpr size_t kTuneOutElems = (size_t)1 << 26;      // 512 MiB of outputs: 4096 tiles of any N <= 8192

// Batch workspace: status words, tile counters, tables, then one update layout per problem.
struct BatchWs {
  int* status;
  int* counters;
  char* tables;
  size_t table_bytes;
  std::vector<size_t> layout_off;
  size_t bytes;
};

bool problem_ok(const svdu_problem& p) {
  const int m = p.m, n = p.n;
  if (m < 1 || n < m) return false;
  if (!p.U || !p.sigma || !p.V || !p.a || !p.b || !p.U_out || !p.sigma_out || !p.V_out) return false;
  if (p.ldu < m || p.ldv < n || p.ldu_out < m || p.ldv_out < n) return false;
  return true;
}

size_t table_bytes_for(int count, const svdu_problem* probs, int precision, const Options& opt) {
  std::vector<Update> ups(count);
  for (int i = 0; i < count; ++i) {
    ups[i].m = probs[i].m;
    ups[i].n = probs[i].n;
    ups[i].defl = probs[i].defl;
    ups[i].L = carve_update(nullptr, probs[i].m, probs[i].n, SVDU_PATH_DIRECT, precision);
  }
  std::vector<char> blob;
  Plan P;
  build_plan(ups, precision, opt, nullptr, nullptr, &blob, &P);
  // the lists per tile shape are padded to 16 bytes each, so the size
  // depends a little on the shapes chosen: leave room for any choice
  return blob.size() + 4096;
}

BatchWs carve_batch(void* ws, int count, const svdu_problem* probs, int precision, size_t table_bytes) {
  BatchWs W;
  Carver c(ws);
  W.status = c.take<int>(count);
  W.counters = c.take<int>(2 * kNumShapes);
  W.tables = c.take<char>(table_bytes);
  W.table_bytes = table_bytes;
  for (int i = 0; i < count; ++i) {
    const size_t lb = carve_update(nullptr, probs[i].m, probs[i].n, SVDU_PATH_DIRECT, precision).bytes;
    c.off = (c.off + 255) & ~size_t(255);
    W.layout_off.push_back(c.off);
    c.off += lb;
  }
  W.bytes = c.off + 256;
  return W;
}

// Memory ranges of a batch; outputs must not overlap each other, any input or
// the workspace.
struct Range {
  uintptr_t lo, hi;
  bool out;
};

bool ranges_ok(std::vector<Range> r) {
  std::sort(r.begin(), r.end(), [](const Range& x, const Range& y) { return x.lo < y.lo; });
  // sweep: track the furthest end so far of outputs and of all ranges
  uintptr_t end_any = 0, end_out = 0;
  bool started = false;
  for (const Range& x : r) {
    if (x.hi <= x.lo) continue;
    if (started) {
      if (x.out && x.lo < end_any) return false;    // an output starts inside an earlier range
      if (!x.out && x.lo < end_out) return false;   // an input starts inside an earlier output
    }
    started = true;
    end_any = std::max(end_any, x.hi);
    if (x.out) end_out = std::max(end_out, x.hi);
  }
  return true;
}

size_t span(int rows, int cols, int ld) { return ((size_t)(rows - 1) * ld + cols) * 8; }

void destroy_graph(svdu_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// ---------------------------------------------------------------------------
// autotuner kernels: synthetic all-live descriptors and operand fill
// ---------------------------------------------------------------------------
__global__ void synth_desc_kernel(int N, double* rg, double* rzeta, double* rh, int* rcl, int8_t* ctype,
                                  double* co, double* ctau, double* ccs, int* ccl, int* cmem, double* ch,
                                  int* status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) status[0] = 0;
  if (j < N) {
    rg[j] = 1.0 + j;
    rzeta[j] = 1.0 / sqrt((double)N);
    rh[j] = 0.0;
    rcl[j] = j;
    ctype[j] = 0;
    co[j] = 1.0 + j;
    ctau[j] = 0.5;
    ccs[j] = 1.0;
    ccl[j] = -1;
    cmem[j] = -1;
    ch[j] = 0.0;
  }
}

__global__ void fill_kernel(size_t n, double* x) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = hash_unit(i, 7);
}

}  // namespace

extern "C" {

size_t svdu_batch_workspace_bytes(int count, const svdu_problem* probs, int precision) {
  if (count < 1 || !probs) return 0;
  if (!precision_ok(precision)) return 0;
  for (int i = 0; i < count; ++i)
    if (!(probs[i].m >= 1 && probs[i].n >= probs[i].m)) return 0;
  const size_t tb = table_bytes_for(count, probs, precision, Options());
  return carve_batch(nullptr, count, probs, precision, tb).bytes;
}

int svdu_batch_create(svdu_ctx* ctx, svdu_batch** out, int count, const svdu_problem* probs, int precision, int flags,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return SVDU_EINVAL;
  *out = nullptr;
  if (!ctx || count < 1 || !probs || !workspace) return SVDU_EINVAL;
  if (!precision_ok(precision)) return SVDU_EINVAL;
  if (flags & ~SVDU_BATCH_PERSISTENT) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!problem_ok(probs[i])) return SVDU_EINVAL;
  for (int i = 0; i < count; ++i)
    if (precision == SVDU_PREC_SLICED_INT8 && probs[i].n > kI8MaxN) return SVDU_ENOTSUP;
  const size_t tb = table_bytes_for(count, probs, precision, Options());
  BatchWs W = carve_batch(workspace, count, probs, precision, tb);
  if (workspace_bytes < W.bytes) return SVDU_ENOMEM;
  {
    std::vector<Range> r;
    r.push_back({reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + W.bytes, true});
    for (int i = 0; i < count; ++i) {
      const svdu_problem& p = probs[i];
      auto add = [&](const void* ptr, size_t bytes, bool o) {
        r.push_back({reinterpret_cast<uintptr_t>(ptr), reinterpret_cast<uintptr_t>(ptr) + bytes, o});
      };
      add(p.U, span(p.m, p.m, p.ldu), false);
      add(p.V, span(p.n, p.n, p.ldv), false);
      add(p.sigma, (size_t)p.m * 8, false);
      add(p.a, (size_t)p.m * 8, false);
      add(p.b, (size_t)p.n * 8, false);
      add(p.U_out, span(p.m, p.m, p.ldu_out), true);
      add(p.V_out, span(p.n, p.n, p.ldv_out), true);
      add(p.sigma_out, (size_t)p.m * 8, true);
      if (p.defl) add(p.defl, (size_t)4 * p.n, true);
    }
    if (!ranges_ok(r)) return SVDU_EINVAL;
  }
  if (const int rc = ctx_device_check(ctx)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  svdu_batch* b = new svdu_batch;
  b->ctx = ctx;
  b->opt = ctx->opt;
  b->count = count;
  b->precision = precision;
  b->persistent = (flags & SVDU_BATCH_PERSISTENT) != 0;
  b->status_dev = W.status;
  b->counters = W.counters;
  b->tables = W.tables;
  b->ups.resize(count);
  for (int i = 0; i < count; ++i) {
    const svdu_problem& p = probs[i];
    Update& u = b->ups[i];
    u.m = p.m;
    u.n = p.n;
    u.U = p.U;
    u.sigma = p.sigma;
    u.V = p.V;
    u.a = p.a;
    u.b = p.b;
    u.ldu = p.ldu;
    u.ldv = p.ldv;
    u.U_out = p.U_out;
    u.sigma_out = p.sigma_out;
    u.V_out = p.V_out;
    u.ldu_out = p.ldu_out;
    u.ldv_out = p.ldv_out;
    u.defl = p.defl;
    u.L = carve_update(static_cast<char*>(workspace) + W.layout_off[i], p.m, p.n, SVDU_PATH_DIRECT, precision);
  }
  std::vector<char> blob;
  build_plan(b->ups, precision, b->opt, W.tables, W.counters, &blob, &b->plan);
  int rc = SVDU_OK;
  if (blob.size() > W.table_bytes) rc = SVDU_ENOMEM;
  if (rc == SVDU_OK && hipHostMalloc(reinterpret_cast<void**>(&b->pinned), std::max<size_t>(blob.size(), 16)) != hipSuccess)
    rc = SVDU_EHIP;
  if (rc == SVDU_OK && hipHostMalloc(reinterpret_cast<void**>(&b->status_host), sizeof(int) * count) != hipSuccess)
    rc = SVDU_EHIP;
  if (rc == SVDU_OK && hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess) rc = SVDU_EHIP;
  if (rc == SVDU_OK) {
    memcpy(b->pinned, blob.data(), blob.size());
    if (hipMemcpyAsync(W.tables, b->pinned, blob.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(b->uploaded, st) != hipSuccess)
      rc = SVDU_EHIP;
  }
  if (rc != SVDU_OK) {
    if (b->uploaded) {
      (void)hipStreamSynchronize(st);
      (void)hipEventDestroy(b->uploaded);
    }
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->status_host) (void)hipHostFree(b->status_host);
    delete b;
    return rc;
  }
  *out = b;
  return SVDU_OK;
}

int svdu_batch_launch(svdu_batch* b, int use_graph, void* stream) {
  if (!b) return SVDU_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamWaitEvent(st, b->uploaded, 0) != hipSuccess) return SVDU_EHIP;
  if (!use_graph) {
    const Sched S = sched_of(b->ctx, b->opt, b->persistent, true);
    enqueue_plan(b->plan, S, kStepAll, st);
    return hipGetLastError() == hipSuccess ? SVDU_OK : SVDU_EHIP;
  }
  if (!b->exec) {
    // capture the whole sequence once on a private stream, then replay it
    if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return SVDU_EHIP;
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return SVDU_EHIP;
    const Sched S = sched_of(b->ctx, b->opt, b->persistent, false);
    enqueue_plan(b->plan, S, kStepAll, b->cap_stream);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      destroy_graph(b);
      return SVDU_EHIP;
    }
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
      destroy_graph(b);
      return SVDU_EHIP;
    }
  }
  return hipGraphLaunch(b->exec, st) == hipSuccess ? SVDU_OK : SVDU_EHIP;
}

int svdu_batch_status(svdu_batch* b, int* status, void* stream) {
  if (!b || !status) return SVDU_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamWaitEvent(st, b->uploaded, 0) != hipSuccess) return SVDU_EHIP;
  enqueue_status_gather(b->plan, b->status_dev, st);
  if (hipMemcpyAsync(b->status_host, b->status_dev, sizeof(int) * b->count, hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return SVDU_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SVDU_EHIP;
  int worst = SVDU_OK;
  for (int i = 0; i < b->count; ++i) {
    status[i] = status_code(b->status_host[i]);
    if (status[i] != SVDU_OK && worst == SVDU_OK) worst = status[i];
  }
  return worst;
}

void svdu_batch_destroy(svdu_batch* b) {
  if (!b) return;
  if (b->uploaded) {
    (void)hipEventSynchronize(b->uploaded);
    (void)hipEventDestroy(b->uploaded);
  }
  destroy_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->status_host) (void)hipHostFree(b->status_host);
  delete b;
}

int svdu_rank1_update_batched(svdu_ctx* ctx, int count, const svdu_problem* probs, int precision, void* workspace,
                              size_t workspace_bytes, void* stream) {
  if (!ctx) return SVDU_EINVAL;
  svdu_batch* b = nullptr;
  int rc = svdu_batch_create(ctx, &b, count, probs, precision, ctx->opt.persistent ? SVDU_BATCH_PERSISTENT : 0,
                             workspace, workspace_bytes, stream);
  if (rc != SVDU_OK) return rc;
  rc = svdu_batch_launch(b, 0, stream);
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess && rc == SVDU_OK) rc = SVDU_EHIP;
  svdu_batch_destroy(b);
  return rc;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
size_t svdu_autotune_workspace_bytes(int max_n) {
  if (max_n < 1) return 0;
  const size_t n = (size_t)max_n;
  Carver c(nullptr);
  c.take<int>(16);
  c.take<double>(8 * n);           // rg rzeta rh co ctau ccs ch (+1 spare)
  c.take<int>(3 * n);              // rcl ccl cmem
  c.take<int8_t>(n);               // ctype
  c.take<double>(n * n);           // X
  c.take<double>(std::max<size_t>(n * n, kTuneOutElems));   // outputs
  c.take<char>(1 << 20);           // tables
  return c.off + 256;
}

int svdu_autotune(svdu_ctx* ctx, int precision, int max_n, double* times_ms, int* table, void* workspace,
                  size_t workspace_bytes, void* stream) {
  if (!ctx) return SVDU_EINVAL;
  if (precision != SVDU_PREC_FP64 && precision != SVDU_PREC_SPLIT32) return SVDU_EINVAL;
  if (max_n < 16 || !workspace) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SVDU_EINVAL;
  if (workspace_bytes < svdu_autotune_workspace_bytes(max_n)) return SVDU_ENOMEM;
  if (const int rc = ctx_device_check(ctx)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)max_n;
  int* tab = ctx->opt.shape_table[precision == SVDU_PREC_SPLIT32 ? 1 : 0];
  Carver c(workspace);
  int* status = c.take<int>(16);
  double* dd = c.take<double>(8 * n);
  int* ii = c.take<int>(3 * n);
  int8_t* ctype = c.take<int8_t>(n);
  double* X = c.take<double>(n * n);
  const size_t out_elems = std::max<size_t>(n * n, kTuneOutElems);
  double* Xo = c.take<double>(out_elems);
  char* tables = c.take<char>(1 << 20);
  CauchyDesc d{};
  double *rg = dd, *rzeta = dd + n, *rh = dd + 2 * n, *co = dd + 3 * n, *ctau = dd + 4 * n, *ccs = dd + 5 * n,
         *ch = dd + 6 * n;
  int *rcl = ii, *ccl = ii + n, *cmem = ii + 2 * n;
  hipLaunchKernelGGL(synth_desc_kernel, dim3(cdiv(max_n, 256)), dim3(256), 0, st, max_n, rg, rzeta, rh, rcl,
                     ctype, co, ctau, ccs, ccl, cmem, ch, status);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, n * n, X);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SVDU_EHIP;
  int rc = SVDU_OK;
  for (int bk = 0; bk < kShapeBuckets && rc == SVDU_OK; ++bk) {
    const int hi = std::min(64 << bk, max_n), lo = bk == 0 ? 0 : (64 << (bk - 1));
    if (bk > 0 && lo >= max_n) {   // bucket beyond max_n: keep the table entry
      if (times_ms)
        for (int s = 0; s < kNumShapes; ++s) times_ms[bk * kNumShapes + s] = -1.0;
      if (table) table[bk] = tab[bk];
      continue;
    }
    // the same set of products for every shape, of kTuneOrders orders spread
    // over the bucket (a shape's ragged last tile row costs differently at
    // different orders), each as many times as make kTuneTiles / kTuneOrders
    // tiles of 128 x 128, so that every shape sees the device full
    std::vector<int> Ns, counts;
    size_t used = 0;
    for (int j = 0; j < kTuneOrders; ++j) {
      const int N = std::max(1, lo + ((hi - lo) * (j + 1) + kTuneOrders - 1) / kTuneOrders);
      const int tiles128 = cdiv(N, 128) * cdiv(N, 128);
      int count = std::max(1, cdiv(kTuneTiles / kTuneOrders, tiles128));
      count = (int)std::min<size_t>((size_t)count, (out_elems - used) / ((size_t)N * N));
      if (count < 1) continue;
      Ns.push_back(N);
      counts.push_back(count);
      used += (size_t)count * N * N;
    }
    double best = 1e30;
    int best_s = tab[bk];
    for (int s = 0; s < kNumShapes; ++s) {
      std::vector<GemmJob> jobs;
      size_t off = 0;
      for (size_t o = 0; o < Ns.size(); ++o) {
        const int N = Ns[o];
        d = CauchyDesc{N, rg, rzeta, rh, rcl, ctype, co, ctau, ccs, ccl, cmem, ch, nullptr, status};
        for (int k = 0; k < counts[o]; ++k) {
          GemmJob J{};
          J.R = N;
          J.ldx = N;
          J.ldo = N;
          J.vec_a = (N % 2) == 0 ? 1 : 0;
          J.shape = run_shape(s, precision == SVDU_PREC_SPLIT32);
          J.tiles_n = cdiv(N, shape_bn(J.shape));
          J.tiles = cdiv(N, shape_bm(J.shape)) * J.tiles_n;
          J.X = X;
          J.Xo = Xo + off;
          J.d = d;
          jobs.push_back(J);
          off += (size_t)N * N;
        }
      }
      std::vector<char> blob;
      BlobWriter B{&blob, tables};
      const GemmList G = build_gemm_list(jobs, nullptr, B);
      blob.resize((blob.size() + 15) & ~size_t(15));
      if (blob.size() > (1u << 20)) {
        rc = SVDU_ENOMEM;
        break;
      }
      write_blob(blob, tables, st);
      float tbest = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0, st);
        if (precision == SVDU_PREC_SPLIT32)
          launch_gemm_split32(G, run_shape(s, true), false, 0, st);
        else
          launch_gemm_f64(G, s, false, 0, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = SVDU_EHIP;
          break;
        }
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        if (rep > 0) tbest = std::min(tbest, t);   // the first run warms up
      }
      if (rc != SVDU_OK) break;
      if (times_ms) times_ms[bk * kNumShapes + s] = tbest;
      if (tbest < best) {
        best = tbest;
        best_s = s;
      }
    }
    if (rc != SVDU_OK) break;
    tab[bk] = best_s;
    if (table) table[bk] = best_s;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == SVDU_OK && hipGetLastError() != hipSuccess) rc = SVDU_EHIP;
  return rc;
}

int svdu_tile_table(svdu_ctx* ctx, int precision, int* table, int set) {
  if (precision != SVDU_PREC_FP64 && precision != SVDU_PREC_SPLIT32) return SVDU_EINVAL;
  if (!ctx || !table) return SVDU_EINVAL;
  int* tab = ctx->opt.shape_table[precision == SVDU_PREC_SPLIT32 ? 1 : 0];
  for (int b = 0; b < kShapeBuckets; ++b) {
    if (set) {
      if (table[b] < 0 || table[b] >= kNumShapes) return SVDU_EINVAL;
    }
  }
  for (int b = 0; b < kShapeBuckets; ++b) {
    if (set)
      tab[b] = table[b];
    else
      table[b] = tab[b];
  }
  return SVDU_OK;
}

}  // extern "C"
