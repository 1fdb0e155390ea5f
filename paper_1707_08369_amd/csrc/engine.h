// The launch sequence of rank-1 SVD updates (Section 6.1 of the paper) over
// job tables: one update (svdu_rank1_update) or many (the batched entry
// points) run the same kernels in the same order, one launch per step for
// all of them.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string.h>

#include <functional>
#include <vector>

#include "../../include/svdu.h"
#include "cauchy_tile.h"
#include "jobs.h"

namespace svdu {

inline bool precision_ok(int p) {
  return p == SVDU_PREC_FP64 || p == SVDU_PREC_SPLIT32 || p == SVDU_PREC_SLICED_INT8;
}

// ---- options of a context (svdu_ctx) -----------------------------------------------
constexpr int kShapeBuckets = 8;   // N in (0,64], (64,128], ..., (4096, inf)
constexpr int kNumPrec = 2;        // tile-shape tables: SVDU_PREC_FP64, SVDU_PREC_SPLIT32 (the INT8
                                   // product has one tile shape)
int shape_bucket(int N);
// The tile shapes the autotuner measured on MI355X, per precision and bucket.
void default_shape_table(int (&t)[kNumPrec][kShapeBuckets]);

struct Options {
  int maxit = 200;                          // secular iteration cap
  int secular_ff = 1;                       // SVDU_OPT_SECULAR_FMM: 0 direct sums, 1 far field above
                                            // order 2048, 2 far field at every order
  bool refine = true;                       // close-cluster refinement of FP64 results
  bool persistent = false;                  // persistent product schedule
  int forced_shape = -1;                    // -1: the table
  int slices = kDefaultSlices;              // slices of the exact-slice INT8 product
  int shape_table[kNumPrec][kShapeBuckets];
  Options() { default_shape_table(shape_table); }
};
int choose_shape(int N, int precision, const Options& o);
int gemm_grid_cap(int shape, int precision);   // blocks resident at once (persistent schedule)

// ---- timing ring ------------------------------------------------------------------
// HIP events at the boundaries of the phases of each recorded call
// (projections | O(n^2) eigen-update work | products, first level | products,
// second level | flags), for up to kRingCalls calls.
constexpr int kRingCalls = 256, kRingEvents = 6;
struct TimingRing {
  bool on = false;
  int count = 0;
  bool made[kRingCalls] = {};
  hipEvent_t ev[kRingCalls][kRingEvents];
  ~TimingRing();
  int begin();                                // call index, or -1 when off or full
  void mark(int call, int k, hipStream_t st);
  int set(bool on);                           // returns the previous state; resets the record
  int read(double* ms, int max_calls);
};

// ---- workspace carving ------------------------------------------------------
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

void carve_stage(Carver& c, Stage& s, int cap);

// Everything one update keeps in its workspace.
struct Layout {
  int* status;
  double* scal;  // [0] beta [1] alpha [2] b.w1 [3] b.w2
  double *p, *q, *t1, *t2, *w1, *w2;
  double *zLp, *yLm, *pL1, *pL2, *zLm, *pL1b, *pL2b, *fL1, *fL2;
  double *zRp, *yRm, *zRm, *pR1b, *pR2b, *fR1, *fR2;
  double *lamLp, *lamRp, *signs;
  double *gemv_pu, *gemv_pv;      // partial sums of the projections through U and V
  double *renorm_u, *renorm_v;    // precision form: column sums of squares
  double *TL, *TR;                // intermediate bases U~ (m x m) and V~ (n x n)
  int8_t *i8A[2], *i8B[2];        // exact-slice INT8 form, left / right side: slices of X and C~
  int *i8ea[2], *i8eb[2];         // their row / column scale exponents
  int kmax, cmax;                 // cluster refinement: gathered columns, cluster records
  int *rf_info, *rf_start, *rf_size, *rf_off, *rf_idx;
  double *rf_Yu, *rf_Yv, *rf_T, *rf_W, *rf_beta;
  Stage st[4];                    // L+, L-, R+, R-
  double* fmm_work;               // FMM path only (the right-hand products; the single eigen-update)
  size_t fmm_elems;
  double* fmm_work_l;             // FMM path: the left-hand products, which run beside the right-hand ones
  size_t fmm_elems_l;
  char* fmm_plan;
  size_t fmm_plan_bytes;
  size_t bytes;
};
Layout carve_update(void* base, int m, int n, int path, int precision);

// One rank-1 update: the caller's device buffers and its workspace layout.
struct Update {
  int m = 0, n = 0;
  const double *U = nullptr, *sigma = nullptr, *V = nullptr, *a = nullptr, *b = nullptr;
  int ldu = 0, ldv = 0;
  double *U_out = nullptr, *sigma_out = nullptr, *V_out = nullptr;
  int ldu_out = 0, ldv_out = 0;
  int8_t* defl = nullptr;
  Layout L;
};

// ---- per-update jobs (projections set-up, singular values, flags) -------------
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

struct ProbJob {
  int m, n;
  int* status;
  double *w1, *w2;
  SetupArgs setup;
  const double *lamL, *fL1, *fL2, *fR1, *fR2;
  double *sigma_out, *signs;
  int8_t* defl;
  const int8_t* flags[4];
  int fN[4];
};

struct ProbList {
  int n = 0;
  int blocks_n = 0;             // ceil(n / 256) blocks per update
  const int* boff_n = nullptr;
  const ProbJob* job = nullptr;
  int* counters = nullptr;      // persistent-schedule tile counters, zeroed by the first kernel
  int ncounters = 0;
};

// Device views of the tables of one launch sequence.
struct Plan {
  int precision = 0;
  bool any_defl = false;
  ProbList prob;
  GemvList gemv;
  StageLevel lev[2];
  GemmList gemm[2][kNumShapes];
  int slices = kDefaultSlices;      // exact-slice INT8 form: slicing and products per level
  SliceXList sx[2];
  SliceCList sc[2];
  I8List i8[2];
  RenormList renorm;
  RefineList refine;
  std::vector<Stage> host_stages;   // per update: L+, L-, R+, R- (host copies, for the FMM path)
};

// Appends arrays to a host blob that will be copied to dev_base; put()
// returns the device address of the array (dev_base may be nullptr when only
// sizing the blob).
struct BlobWriter {
  std::vector<char>* b;
  char* base;
  template <class T>
  const T* put(const std::vector<T>& v) {
    const size_t off = (b->size() + 15) & ~size_t(15);
    b->resize(off + v.size() * sizeof(T));
    if (!v.empty()) memcpy(b->data() + off, v.data(), v.size() * sizeof(T));
    return reinterpret_cast<const T*>(reinterpret_cast<uintptr_t>(base) + off);
  }
};

// A level of eigen-updates (largest first) with its block offsets.
StageLevel build_level(const std::vector<Stage>& st, const std::vector<TmvJob>& tmv, BlobWriter& B);
// A product job in the tile shape the chooser gives for (R, N, precision).
GemmJob make_gemm_job(int R, const double* X, int ldx, const CauchyDesc& d, double* Xo, int ldo, int precision,
                      const Options& opt);
// A list of products of one tile shape, largest first.
GemmList build_gemm_list(std::vector<GemmJob> jobs, int* counter, BlobWriter& B);

// Tables of `ups` appended to `blob`, with device views relative to
// dev_base (the device address the blob will be copied to; nullptr to size
// the blob only). `counters` points at 2 * kNumShapes ints of device memory.
void build_plan(const std::vector<Update>& ups, int precision, const Options& opt, char* dev_base, int* counters,
                std::vector<char>* blob, Plan* plan);

// Bytes reserved in a single update's workspace for its tables.
constexpr size_t kSingleTableBytes = 16384;

// Copies a host blob to device memory with kernels whose arguments carry the
// bytes (stream-ordered, safe to capture in a graph; no host buffer needs to
// outlive the call).
void write_blob(const std::vector<char>& blob, char* dst, hipStream_t st);

// Step groups of the launch sequence.
enum : int { kStepAll = 0, kStepUpToRoots = 1, kStepProductsOnward = 2 };
struct Sched {
  int maxit = 200;
  int secular_ff = 1;
  bool persistent = false;
  bool refine = true;
  int grid_cap[kNumPrec][kNumShapes] = {};   // [precision][shape]
  TimingRing* ring = nullptr;                // phase events of call `tcall` (nullptr: none)
  int tcall = -1;
  void mark(int k, hipStream_t st) const {
    if (ring) ring->mark(tcall, k, st);
  }
};
// Enqueues the sequence (or a part of it: the FMM path runs the products
// itself between the two parts). after_level, when given, is called once the
// work of each eigen-update level is enqueued (level 0, then 1).
void enqueue_plan(const Plan& P, const Sched& S, int part, hipStream_t st,
                  const std::function<void(int)>* after_level = nullptr);

// Gathers the status words of the plan's updates into out[0..n-1] (device).
void enqueue_status_gather(const Plan& P, int* out, hipStream_t st);

int status_code(int bits);

}  // namespace svdu

// A context: the options, tile tables and timing ring of the calls made with
// it, bound to one device. Every context is independent of the others; one
// context is used by one host thread at a time.
struct svdu_ctx {
  int device = 0;
  svdu::Options opt;
  svdu::TimingRing ring;
  bool have_caps = false;
  int grid_cap[svdu::kNumPrec][svdu::kNumShapes] = {};
  // two more streams for the FMM path's products (default priority), forked
  // from and joined to the caller's stream with events; all are created on
  // first use
  hipStream_t aux = nullptr, aux2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t roots[2] = {nullptr, nullptr};   // the FMM path's root copies of each level are done
  hipEvent_t up0 = nullptr;                   // the first level's plans are uploaded (on aux)
  hipEvent_t done_a = nullptr, done_b = nullptr;   // the first level's products are done (aux, aux2)
  hipEvent_t uploaded = nullptr;              // every plan upload of the last call has read the pinned memory
  bool upload_pending = false;
  // pinned host memory for the FMM path's copies of the roots (grown on
  // demand; every copy into it has completed when a call returns)
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  ~svdu_ctx();
};

namespace svdu {
// The schedule of a call made with `ctx` (queries the device's capacity for
// persistent blocks once per context when `persistent`); `timed`: record the
// call's phases in the context's ring when it is on.
Sched sched_of(svdu_ctx* ctx, const Options& o, bool persistent, bool timed);
// SVDU_OK when the context's device is current, else SVDU_EINVAL (SVDU_EHIP
// when the runtime cannot tell).
int ctx_device_check(const svdu_ctx* ctx);
}  // namespace svdu
