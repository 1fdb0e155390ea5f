// Serving runtime: rank-1 updates of resident matrices, admitted by memory
// and batched as they arrive (continuous batching).
//
// Each registered matrix keeps its factors U, sigma, V in HBM in two buffer
// sets; an update reads the current set and writes the other, which then
// becomes current. Requests carry a release time on the server clock. S
// worker threads, each with its own stream, repeatedly take the oldest
// released request whose matrix is idle and add further released requests
// of a similar size (oldest first, at most one per matrix, cost between
// min_cost_ratio times the first's and the first's, total cost bounded) whose
// workspace fits in the server's device arena (memory admission), so that
// small requests are not held up inside a batch of large ones but go to
// another worker; the batch then runs through the same launch sequence as
// svdu_batch_launch while the other workers keep forming and running
// batches, so work admitted later overlaps work already on the device.
// Updates of one matrix are applied in release order.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/svdu.h"
#include "engine.h"
#include "fmm_tree.h"

using namespace svdu;

namespace {

// First-fit allocator over one device buffer, 256-byte granules, coalescing.
class Arena {
 public:
  void init(char* base, size_t bytes) {
    base_ = base;
    free_.clear();
    free_[0] = bytes & ~size_t(255);
    total_ = free_[0];
  }
  // offset of a block of `bytes`, or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  size_t largest_free() const {
    size_t b = 0;
    for (auto& f : free_) b = std::max(b, f.second);
    return b;
  }
  size_t total() const { return total_; }
  char* base() const { return base_; }

 private:
  char* base_ = nullptr;
  size_t total_ = 0;
  std::map<size_t, size_t> free_, used_;
};

struct Matrix {
  int m = 0, n = 0;
  double* U[2] = {};
  double* s[2] = {};
  double* V[2] = {};
  int cur = 0;
  bool busy = false;
  long long updates = 0;
};

struct Request {
  long long id;
  int matrix;
  const double* a;
  const double* b;
  double t_release;
  double t_start = 0, t_done = 0;
  int status = 0;
  int batch = 0;
  int path = SVDU_PATH_DIRECT;
};

// Workspace of a batch: kBatchFixed bytes (status words, tile counters, the
// base of the tables) plus, per update, its layout and kTableShare bytes of
// tables (an update's job-table entries take about 3 KiB).
constexpr size_t kBatchFixed = 16384, kTableShare = 4096;
size_t update_ws_bytes(int m, int n, int path, int precision) {
  if (path == SVDU_PATH_FMM) return svdu_workspace_bytes(m, n, path, precision) + 256;
  return carve_update(nullptr, m, n, SVDU_PATH_DIRECT, precision).bytes + kTableShare + 256;
}

double cost_of(int m, int n) { return 4.0 * ((double)m * m * m + (double)n * n * n); }

}  // namespace

struct svdu_server {
  svdu_server_config cfg{};
  Options opt;                          // the context's options when the server was created
  int device = 0;
  char* arena_mem = nullptr;
  Arena arena;
  std::vector<Matrix> mats;
  std::deque<Request> pending;          // by release time
  std::vector<svdu_completion> done;
  std::mutex mu;
  std::condition_variable cv;
  bool stopping = false;
  int running = 0;                      // batches on the device
  long long next_id = 0;
  long long batches = 0, batched_updates = 0;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;
  int first_error = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker_main(int w);
};

namespace {

struct Picked {
  std::vector<Request> reqs;
  size_t ws_off = SIZE_MAX, ws_bytes = 0;
};

// Forms a batch from the released, admissible requests (lock held). Returns
// false when nothing can start now.
bool form_batch(svdu_server* S, double now, Picked* out) {
  const svdu_server_config& c = S->cfg;
  auto fmm_of = [&](const Matrix& M) {
    return c.fmm_min_n > 0 && M.n >= c.fmm_min_n && c.precision == SVDU_PREC_FP64;
  };
  // head: the oldest released request whose matrix is idle
  size_t head = SIZE_MAX;
  for (size_t i = 0; i < S->pending.size(); ++i) {
    const Request& r = S->pending[i];
    if (r.t_release > now) break;
    if (!S->mats[r.matrix].busy) {
      head = i;
      break;
    }
  }
  if (head == SIZE_MAX) return false;
  const Matrix& H = S->mats[S->pending[head].matrix];
  const bool hf = fmm_of(H);
  const size_t hws = update_ws_bytes(H.m, H.n, hf ? SVDU_PATH_FMM : SVDU_PATH_DIRECT, c.precision);
  if (hws + kBatchFixed > S->arena.total()) {
    // can never run: complete it with an error
    Request r = S->pending[head];
    S->pending.erase(S->pending.begin() + head);
    r.status = SVDU_ENOMEM;
    r.t_start = r.t_done = now;
    S->done.push_back(svdu_completion{r.id, r.matrix, r.status, 0, r.t_release, r.t_start, r.t_done});
    S->cv.notify_all();
    return false;
  }
  const size_t avail = S->arena.largest_free();
  if (hws + kBatchFixed > avail) return false;   // memory admission: wait for running work to free the arena
  std::vector<size_t> take = {head};
  size_t ws = hws + kBatchFixed;
  if (!hf) {
    const double hc = cost_of(H.m, H.n);
    double tot = hc;
    const double cap = std::max(c.batch_cost_factor * hc, c.min_batch_cost);
    std::vector<int> in_batch = {S->pending[head].matrix};
    for (size_t i = head + 1; i < S->pending.size() && (int)take.size() < c.max_batch; ++i) {
      const Request& r = S->pending[i];
      if (r.t_release > now) break;
      const Matrix& M = S->mats[r.matrix];
      if (M.busy || fmm_of(M)) continue;
      if (std::find(in_batch.begin(), in_batch.end(), r.matrix) != in_batch.end()) continue;
      const double rc = cost_of(M.m, M.n);
      if (rc > hc || rc < c.min_cost_ratio * hc || tot + rc > cap) continue;
      const size_t rws = update_ws_bytes(M.m, M.n, SVDU_PATH_DIRECT, c.precision);
      if (ws + rws > avail) continue;
      take.push_back(i);
      in_batch.push_back(r.matrix);
      tot += rc;
      ws += rws;
    }
  }
  out->ws_off = S->arena.alloc(ws);
  if (out->ws_off == SIZE_MAX) return false;
  out->ws_bytes = ws;
  std::sort(take.begin(), take.end());
  for (size_t k = take.size(); k-- > 0;) {
    Request r = S->pending[take[k]];
    r.path = hf ? SVDU_PATH_FMM : SVDU_PATH_DIRECT;
    out->reqs.push_back(r);
    S->pending.erase(S->pending.begin() + take[k]);
  }
  std::reverse(out->reqs.begin(), out->reqs.end());
  for (Request& r : out->reqs) {
    S->mats[r.matrix].busy = true;
    r.t_start = now;
    r.batch = (int)out->reqs.size();
  }
  return true;
}

}  // namespace

void svdu_server::worker_main(int w) {
  (void)hipSetDevice(device);
  // a private context per worker (for the FMM requests), holding the server's options
  svdu_ctx wctx;
  wctx.device = device;
  wctx.opt = opt;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    if (!first_error) first_error = SVDU_EHIP;
    return;
  }
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  int* status_host = nullptr;
  int status_cap = 0;
  std::vector<char> blob;
  while (true) {
    Picked P;
    {
      std::unique_lock<std::mutex> lk(mu);
      while (true) {
        if (stopping) goto out;
        const double t = now();
        if (form_batch(this, t, &P)) break;
        // sleep until the next release, a completion, or a new request
        double next = -1.0;
        for (const Request& r : pending)
          if (r.t_release > t) {
            next = r.t_release;
            break;
          }
        if (next > 0)
          cv.wait_for(lk, std::chrono::duration<double>(std::min(next - t, 0.05)));
        else
          cv.wait_for(lk, std::chrono::milliseconds(50));
      }
      ++running;
    }
    // run the batch (no lock held)
    char* ws = arena.base() + P.ws_off;
    const int cnt = (int)P.reqs.size();
    std::vector<int> st_codes(cnt, SVDU_OK);
    int rc = SVDU_OK;
    if (P.reqs[0].path == SVDU_PATH_FMM) {
      const Request& r = P.reqs[0];
      Matrix& M = mats[r.matrix];
      const int c0 = M.cur, c1 = 1 - M.cur;
      rc = svdu_rank1_update(&wctx, M.m, M.n, M.U[c0], M.m, M.s[c0], M.V[c0], M.n, r.a, r.b, cfg.fmm_eps,
                             SVDU_PATH_FMM,
                             SVDU_PREC_FP64, M.U[c1], M.m, M.s[c1], M.V[c1], M.n, nullptr, ws, P.ws_bytes, st);
      if (rc == SVDU_OK) rc = svdu_get_status(ws, st);
      st_codes[0] = rc;
    } else {
      // tables at the start of the region, then one layout per update
      Carver c(ws);
      int* status_dev = c.take<int>(cnt);
      int* counters = c.take<int>(2 * kNumShapes);
      const size_t table_bytes = kTableShare * cnt + 4096;
      char* tables = c.take<char>(table_bytes);
      std::vector<Update> ups(cnt);
      for (int i = 0; i < cnt; ++i) {
        const Request& r = P.reqs[i];
        Matrix& M = mats[r.matrix];
        const int c0 = M.cur, c1 = 1 - M.cur;
        Update& u = ups[i];
        u.m = M.m;
        u.n = M.n;
        u.U = M.U[c0];
        u.sigma = M.s[c0];
        u.V = M.V[c0];
        u.a = r.a;
        u.b = r.b;
        u.ldu = M.m;
        u.ldv = M.n;
        u.U_out = M.U[c1];
        u.sigma_out = M.s[c1];
        u.V_out = M.V[c1];
        u.ldu_out = M.m;
        u.ldv_out = M.n;
        u.defl = nullptr;
        c.off = (c.off + 255) & ~size_t(255);
        u.L = carve_update(ws + c.off, M.m, M.n, SVDU_PATH_DIRECT, cfg.precision);
        c.off += u.L.bytes;
      }
      if (c.off > P.ws_bytes) rc = SVDU_ENOMEM;
      blob.clear();
      Plan plan;
      if (rc == SVDU_OK) {
        build_plan(ups, cfg.precision, opt, tables, counters, &blob, &plan);
        if (blob.size() > table_bytes) rc = SVDU_ENOMEM;
      }
      if (rc == SVDU_OK && blob.size() > pinned_bytes) {
        if (pinned) (void)hipHostFree(pinned);
        pinned_bytes = std::max(blob.size(), (size_t)65536);
        if (hipHostMalloc(reinterpret_cast<void**>(&pinned), pinned_bytes) != hipSuccess) {
          pinned = nullptr;
          pinned_bytes = 0;
          rc = SVDU_EHIP;
        }
      }
      if (rc == SVDU_OK && cnt > status_cap) {
        if (status_host) (void)hipHostFree(status_host);
        status_cap = std::max(cnt, 64);
        if (hipHostMalloc(reinterpret_cast<void**>(&status_host), sizeof(int) * status_cap) != hipSuccess) {
          status_host = nullptr;
          status_cap = 0;
          rc = SVDU_EHIP;
        }
      }
      if (rc == SVDU_OK) {
        memcpy(pinned, blob.data(), blob.size());
        if (hipMemcpyAsync(tables, pinned, blob.size(), hipMemcpyHostToDevice, st) != hipSuccess) rc = SVDU_EHIP;
      }
      if (rc == SVDU_OK) {
        enqueue_plan(plan, sched_of(nullptr, opt, false, false), kStepAll, st);
        enqueue_status_gather(plan, status_dev, st);
        if (hipMemcpyAsync(status_host, status_dev, sizeof(int) * cnt, hipMemcpyDeviceToHost, st) != hipSuccess)
          rc = SVDU_EHIP;
      }
      if (hipStreamSynchronize(st) != hipSuccess && rc == SVDU_OK) rc = SVDU_EHIP;
      for (int i = 0; i < cnt; ++i) st_codes[i] = (rc == SVDU_OK) ? status_code(status_host[i]) : rc;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      const double t = now();
      for (int i = 0; i < cnt; ++i) {
        Request& r = P.reqs[i];
        Matrix& M = mats[r.matrix];
        r.status = st_codes[i];
        r.t_done = t;
        if (r.status == SVDU_OK) {   // the other buffer set now holds the factors
          M.cur = 1 - M.cur;
          ++M.updates;
        }
        M.busy = false;
        done.push_back(svdu_completion{r.id, r.matrix, r.status, r.batch, r.t_release, r.t_start, r.t_done});
      }
      arena.release(P.ws_off);
      ++batches;
      batched_updates += cnt;
      --running;
      if (rc != SVDU_OK && !first_error) first_error = rc;
    }
    cv.notify_all();
  }
out:
  if (pinned) (void)hipHostFree(pinned);
  if (status_host) (void)hipHostFree(status_host);
  (void)hipStreamDestroy(st);
}

extern "C" {

int svdu_server_create(svdu_ctx* ctx, svdu_server** out, const svdu_server_config* cfg, void* arena,
                       size_t arena_bytes) {
  if (!out || !ctx || !cfg || !arena) return SVDU_EINVAL;
  *out = nullptr;
  if (cfg->workers < 1 || cfg->workers > 8 || cfg->max_batch < 1) return SVDU_EINVAL;
  if (!precision_ok(cfg->precision)) return SVDU_EINVAL;
  if (cfg->fmm_min_n > 0 && !(cfg->fmm_eps > 0.0 && cfg->fmm_eps < 1.0)) return SVDU_EINVAL;
  if (cfg->fmm_min_n > 0 && fmm_required_order(cfg->fmm_eps) > kFmmMaxOrder) return SVDU_ENOTSUP;
  if (!(cfg->batch_cost_factor >= 1.0) || cfg->min_batch_cost < 0.0) return SVDU_EINVAL;
  if (!(cfg->min_cost_ratio >= 0.0 && cfg->min_cost_ratio <= 1.0)) return SVDU_EINVAL;
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0 || arena_bytes < (1u << 20)) return SVDU_EINVAL;
  if (const int rc = ctx_device_check(ctx)) return rc;
  svdu_server* S = new svdu_server;
  S->cfg = *cfg;
  S->opt = ctx->opt;
  S->device = ctx->device;
  S->arena_mem = static_cast<char*>(arena);
  S->arena.init(S->arena_mem, arena_bytes);
  S->t0 = std::chrono::steady_clock::now();
  *out = S;
  return SVDU_OK;
}

int svdu_server_add_matrix(svdu_server* S, int m, int n, double* U0, double* s0, double* V0, double* U1, double* s1,
                           double* V1, int* id) {
  if (!S || !id || m < 1 || n < m || !U0 || !s0 || !V0 || !U1 || !s1 || !V1) return SVDU_EINVAL;
  if (S->cfg.precision == SVDU_PREC_SLICED_INT8 && n > kI8MaxN) return SVDU_ENOTSUP;
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->workers.empty()) return SVDU_EINVAL;   // matrices are registered before start
  Matrix M;
  M.m = m;
  M.n = n;
  M.U[0] = U0;
  M.s[0] = s0;
  M.V[0] = V0;
  M.U[1] = U1;
  M.s[1] = s1;
  M.V[1] = V1;
  S->mats.push_back(M);
  *id = (int)S->mats.size() - 1;
  return SVDU_OK;
}

int svdu_server_start(svdu_server* S) {
  if (!S) return SVDU_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->workers.empty()) return SVDU_EINVAL;
  S->t0 = std::chrono::steady_clock::now();
  for (int w = 0; w < S->cfg.workers; ++w) S->workers.emplace_back(&svdu_server::worker_main, S, w);
  return SVDU_OK;
}

double svdu_server_now(svdu_server* S) { return S ? S->now() : 0.0; }

int svdu_server_submit(svdu_server* S, int matrix, const double* a, const double* b, double t_release,
                       long long* req_id) {
  if (!S || !a || !b) return SVDU_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (matrix < 0 || matrix >= (int)S->mats.size()) return SVDU_EINVAL;
    Request r;
    r.id = S->next_id++;
    r.matrix = matrix;
    r.a = a;
    r.b = b;
    r.t_release = t_release;
    // keep `pending` ordered by release time (stable for equal times)
    auto it = S->pending.end();
    while (it != S->pending.begin() && std::prev(it)->t_release > t_release) --it;
    S->pending.insert(it, r);
    if (req_id) *req_id = r.id;
  }
  S->cv.notify_all();
  return SVDU_OK;
}

int svdu_server_poll(svdu_server* S, svdu_completion* out, int max_out) {
  if (!S || (!out && max_out > 0)) return SVDU_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  const int n = std::min<int>(max_out, (int)S->done.size());
  for (int i = 0; i < n; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + n);
  return n;
}

int svdu_server_stats(svdu_server* S, long long* stats) {
  if (!S || !stats) return SVDU_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  stats[0] = (long long)S->pending.size();
  stats[1] = S->running;
  stats[2] = S->batches;
  stats[3] = S->batched_updates;
  stats[4] = (long long)S->arena.largest_free();
  stats[5] = S->first_error;
  return SVDU_OK;
}

int svdu_server_drain(svdu_server* S, double timeout_s) {
  if (!S) return SVDU_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (!S->pending.empty() || S->running > 0) {
    if (S->workers.empty()) return SVDU_EINVAL;
    if (S->cv.wait_until(lk, until) == std::cv_status::timeout) return SVDU_ENOCONV;
  }
  return S->first_error;
}

int svdu_server_current(svdu_server* S, int matrix, double** U, double** sigma, double** V) {
  if (!S) return SVDU_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (matrix < 0 || matrix >= (int)S->mats.size()) return SVDU_EINVAL;
  const Matrix& M = S->mats[matrix];
  if (M.busy) return SVDU_EINVAL;
  if (U) *U = M.U[M.cur];
  if (sigma) *sigma = M.s[M.cur];
  if (V) *V = M.V[M.cur];
  return SVDU_OK;
}

void svdu_server_destroy(svdu_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv.notify_all();
  for (std::thread& t : S->workers) t.join();
  delete S;
}

}  // extern "C"
