// Launch sequence of rank-1 SVD updates over job tables (see engine.h).
//
// Device work, all on one stream, each step one launch for every update:
//   1. status words, probes w1 and w2; projections p = U^T a and
//      [q t1 t2] = V^T [b w1 w2] (Algorithm Step 1 / RankOneUpdate Step 1);
//   2. the 2x2 splits (Algorithm Steps 2-3) and every projected vector in
//      core space: U^T a1 = q11 p + q21 S q, U^T b1 = q12 p + q22 S q, and the
//      same on the right with S^T p; validation of the inputs (a non-finite
//      entry of U or V shows up as a non-finite projection);
//   3. the eigen-updates (Steps 4-7) in two levels, (L+, R+) then (L-, R-):
//      deflation, secular roots, weights, descriptors of C~; the second update
//      of each side gets its z as C~^T (U^T b1) of the first;
//   4. singular values (Step 8) and the signs that pair V^ with U^ (not in
//      the paper): s_i = sign((U^T A^ w)_i (V^T w)_i) from two probes mapped
//      through the C~^T of both updates;
//   5. the products X C~ (Steps 4-7) in two levels, (U C~_L+, V C~_R+) then
//      (U~ C~_L-, V~ C~_R- diag(s)); the precision form then rescales the
//      columns of U^ and V^;
//   6. the deflation flags.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>

#include "../../include/svdu.h"
#include "device_util.h"
#include "engine.h"

namespace svdu {

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------
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

Layout carve_update(void* base, int m, int n, int path, int precision) {
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
  L.gemv_pu = c.take<double>(gemv_t_scratch_elems(m, m, 1));
  L.gemv_pv = c.take<double>(gemv_t_scratch_elems(n, n, 3));
  const bool s32 = precision == SVDU_PREC_SPLIT32;
  L.renorm_u = c.take<double>(s32 ? renorm_scratch_elems(m, m) : 0);
  L.renorm_v = c.take<double>(s32 ? renorm_scratch_elems(n, n) : 0);
  for (int k = 0; k < 4; ++k) carve_stage(c, L.st[k], k < 2 ? m : n);
  const bool fmm = path == SVDU_PATH_FMM;
  L.TL = c.take<double>((size_t)m * m);
  L.TR = c.take<double>((size_t)n * n);
  const bool i8 = precision == SVDU_PREC_SLICED_INT8;
  for (int k = 0; k < 2; ++k) {
    const size_t N = (size_t)(k == 0 ? m : n);
    const size_t Rp = i8_pad((int)N, kI8BM), Kp = i8_pad((int)N, kI8K), Cp = i8_pad((int)N, kI8BN);
    L.i8A[k] = c.take<int8_t>(i8 ? kMaxSlices * Rp * Kp : 0);
    L.i8B[k] = c.take<int8_t>(i8 ? kMaxSlices * Cp * Kp : 0);
    L.i8ea[k] = c.take<int>(i8 ? Rp : 0);
    L.i8eb[k] = c.take<int>(i8 ? Cp : 0);
  }
  L.kmax = std::min(m, 128);
  L.cmax = std::max(1, L.kmax / 2);
  const bool rf = precision != SVDU_PREC_SPLIT32;   // refinement of FP64-accurate results
  const size_t km = rf ? (size_t)L.kmax : 0;
  L.rf_info = c.take<int>(4);
  L.rf_start = c.take<int>(rf ? L.cmax : 0);
  L.rf_size = c.take<int>(rf ? L.cmax : 0);
  L.rf_off = c.take<int>(rf ? L.cmax : 0);
  L.rf_idx = c.take<int>(km);
  L.rf_Yu = c.take<double>(km * m);
  L.rf_Yv = c.take<double>(km * n);
  L.rf_T = c.take<double>(km * m);
  L.rf_W = c.take<double>(km * m);
  L.rf_beta = c.take<double>(km);
  L.fmm_elems = fmm ? fmm_workspace_elems(n, n) : 0;
  L.fmm_work = c.take<double>(L.fmm_elems);
  L.fmm_elems_l = fmm ? fmm_workspace_elems(m, m) : 0;
  L.fmm_work_l = c.take<double>(L.fmm_elems_l);
  L.fmm_plan_bytes = fmm ? 4 * fmm_plan_bytes(n) : 0;
  L.fmm_plan = c.take<char>(L.fmm_plan_bytes);
  L.bytes = c.off + 256;
  return L;
}

// ---------------------------------------------------------------------------
// per-update kernels
// ---------------------------------------------------------------------------
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

__device__ void setup_body(const SetupArgs& A) {
  __shared__ double sh[64];
  const int m = A.m, n = A.n, tid = threadIdx.x, nt = blockDim.x;
  double bb = 0.0, aa = 0.0, bw1 = 0.0, bw2 = 0.0;
  int bad = 0;
  for (int j = tid; j < n; j += nt) {
    const double bj = A.b[j];
    bb += bj * bj;
    bw1 += bj * A.w1[j];
    bw2 += bj * A.w2[j];
    if (!isfinite(bj) || !isfinite(A.q[j]) || !isfinite(A.t1[j]) || !isfinite(A.t2[j])) bad |= kStNonFinite;
  }
  for (int j = tid; j < m; j += nt) {
    const double aj = A.a[j], sj = A.sigma[j];
    aa += aj * aj;
    if (!isfinite(aj) || !isfinite(sj) || !isfinite(A.p[j])) bad |= kStNonFinite;
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

__global__ __launch_bounds__(256) void prob_init_kernel(ProbList P) {
  const int u = find_job(P.boff_n, P.n, blockIdx.x);
  const ProbJob J = P.job[u];
  const int j = (blockIdx.x - P.boff_n[u]) * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < P.ncounters) P.counters[threadIdx.x] = 0;
  if (j == 0) J.status[0] = 0;
  if (j < J.n) {
    J.w1[j] = hash_unit((uint64_t)j, 1);
    J.w2[j] = hash_unit((uint64_t)j, 2);
  }
}

__global__ __launch_bounds__(1024) void prob_setup_kernel(ProbList P) {
  const ProbJob& J = P.job[blockIdx.x];
  const SetupArgs A = J.setup;
  setup_body(A);
}

__global__ __launch_bounds__(256) void prob_finalize_kernel(ProbList P) {
  const int u = find_job(P.boff_n, P.n, blockIdx.x);
  const ProbJob J = P.job[u];
  const int i = (blockIdx.x - P.boff_n[u]) * 256 + threadIdx.x;
  if (i < J.m) {
    J.sigma_out[i] = sqrt(fmax(J.lamL[i], 0.0));
    const double p1 = J.fL1[i] * J.fR1[i], p2 = J.fL2[i] * J.fR2[i];
    const double p = (fabs(p1) >= fabs(p2)) ? p1 : p2;
    J.signs[i] = (p < 0.0) ? -1.0 : 1.0;
  } else if (i < J.n) {
    J.signs[i] = 1.0;
  }
}

// Copies the four rows of flags of an update into defl (4 x n), zero-filling
// each row beyond its eigen-update's dimension.
__global__ __launch_bounds__(256) void prob_flags_kernel(ProbList P) {
  const int u = find_job(P.boff_n, P.n, blockIdx.x);
  const ProbJob J = P.job[u];
  if (!J.defl) return;
  const int j = (blockIdx.x - P.boff_n[u]) * 256 + threadIdx.x;
  if (j >= J.n) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) J.defl[(size_t)k * J.n + j] = (j < J.fN[k]) ? J.flags[k][j] : (int8_t)0;
}

__global__ void prob_status_kernel(ProbList P, int* out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < P.n) out[u] = P.job[u].status[0];
}

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
namespace {

std::vector<int> prefix(const std::vector<int>& blocks) {
  std::vector<int> o(blocks.size() + 1, 0);
  for (size_t i = 0; i < blocks.size(); ++i) o[i + 1] = o[i] + blocks[i];
  return o;
}

int cdiv(int a, int b) { return (a + b - 1) / b; }

bool aligned16(const void* p, int ld) { return (ld % 2) == 0 && (reinterpret_cast<uintptr_t>(p) % 16) == 0; }

void stage_inputs(Update& u) {
  Layout& L = u.L;
  Stage& sLp = L.st[0];
  Stage& sLm = L.st[1];
  Stage& sRp = L.st[2];
  Stage& sRm = L.st[3];
  for (int k = 0; k < 4; ++k) L.st[k].status = L.status;
  sLp.N = u.m; sLp.lam_in = L.lamLp; sLp.z = L.zLp; sLp.descending = false;
  sLm.N = u.m; sLm.lam_in = sLp.lam_out; sLm.z = L.zLm; sLm.descending = true;
  sRp.N = u.n; sRp.lam_in = L.lamRp; sRp.z = L.zRp; sRp.descending = false;
  sRm.N = u.n; sRm.lam_in = sRp.lam_out; sRm.z = L.zRm; sRm.descending = true;
}

}  // namespace

StageLevel build_level(const std::vector<Stage>& st_in, const std::vector<TmvJob>& tv_in, BlobWriter& B) {
  std::vector<int> order(st_in.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return st_in[x].N > st_in[y].N; });
  std::vector<Stage> st;
  std::vector<TmvJob> tv;
  std::vector<int> bw, bt, bs, bq, bl;
  for (int i : order) {
    st.push_back(st_in[i]);
    tv.push_back(i < (int)tv_in.size() ? tv_in[i] : TmvJob{0, {nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}});
    bw.push_back(cdiv(st_in[i].N, 4));
    bt.push_back(cdiv(st_in[i].N, 256));
    bs.push_back(st_in[i].N <= kGroupMaxN ? cdiv(st_in[i].N, 256 / kSmallGroup) : cdiv(st_in[i].N, 4));
    bq.push_back(cdiv(bs.back(), 4));
    bl.push_back(cdiv(st_in[i].N, kSfLeaf) + 1);   // leaves, then the extreme root
  }
  const std::vector<int> ow = prefix(bw), ot = prefix(bt), os = prefix(bs), oq = prefix(bq), ol = prefix(bl);
  StageLevel S;
  S.n = (int)st.size();
  S.st = B.put(st);
  S.tmv = B.put(tv);
  S.boff_w = B.put(ow);
  S.boff_t = B.put(ot);
  S.boff_i = B.put(os);
  S.boff_s = B.put(oq);
  S.boff_l = B.put(ol);
  S.blocks_w = ow.back();
  S.blocks_t = ot.back();
  S.blocks_i = os.back();
  S.blocks_s = oq.back();
  S.blocks_l = ol.back();
  for (const Stage& x : st) S.nmax = std::max(S.nmax, x.N);
  return S;
}

GemmJob make_gemm_job(int R, const double* X, int ldx, const CauchyDesc& d, double* Xo, int ldo, int precision,
                      const Options& opt) {
  const int sh = run_shape(choose_shape(d.N, precision, opt), precision == SVDU_PREC_SPLIT32);
  GemmJob J{};
  J.R = R;
  J.ldx = ldx;
  J.ldo = ldo;
  J.vec_a = aligned16(X, ldx) ? 1 : 0;
  J.shape = sh;
  J.tiles_n = cdiv(d.N, shape_bn(sh));
  J.tiles = cdiv(R, shape_bm(sh)) * J.tiles_n;
  J.X = X;
  J.Xo = Xo;
  J.d = d;
  return J;
}

GemmList build_gemm_list(std::vector<GemmJob> jobs, int* counter, BlobWriter& B) {
  jobs.erase(std::remove_if(jobs.begin(), jobs.end(), [](const GemmJob& j) { return j.R <= 0 || j.d.N <= 0; }),
             jobs.end());
  std::stable_sort(jobs.begin(), jobs.end(), [](const GemmJob& x, const GemmJob& y) {
    return (double)x.R * x.d.N * x.d.N > (double)y.R * y.d.N * y.d.N;
  });
  std::vector<int> bl;
  for (const GemmJob& j : jobs) bl.push_back(j.tiles);
  const std::vector<int> o = prefix(bl);
  GemmList G;
  G.n = (int)jobs.size();
  G.blocks = o.back();
  G.boff = B.put(o);
  G.job = B.put(jobs);
  G.counter = counter;
  for (const GemmJob& j : jobs) G.copy |= (j.d.Llist != nullptr) ? 1 : 0;
  return G;
}

void build_plan(const std::vector<Update>& ups_in, int precision, const Options& opt, char* dev_base, int* counters,
                std::vector<char>* blob, Plan* plan) {
  std::vector<Update> ups = ups_in;
  for (Update& u : ups) stage_inputs(u);
  BlobWriter B{blob, dev_base};
  Plan& P = *plan;
  P.precision = precision;
  P.any_defl = false;
  P.host_stages.clear();
  const int nu = (int)ups.size();

  // per-update jobs
  {
    std::vector<ProbJob> jobs(nu);
    std::vector<int> bn(nu);
    for (int i = 0; i < nu; ++i) {
      const Update& u = ups[i];
      const Layout& L = u.L;
      ProbJob& J = jobs[i];
      memset(&J, 0, sizeof(J));
      J.m = u.m;
      J.n = u.n;
      J.status = L.status;
      J.w1 = L.w1;
      J.w2 = L.w2;
      J.setup = SetupArgs{u.m,        u.n,        u.sigma,    u.a,        u.b,      L.p,      L.q,
                          L.t1,       L.t2,       L.w1,       L.w2,       L.scal,   L.status, L.st[0].rho,
                          L.st[1].rho, L.st[2].rho, L.st[3].rho, L.zLp,    L.yLm,    L.pL1,    L.pL2,
                          L.lamLp,    L.zRp,      L.yRm,      L.lamRp,    L.st[0].col_of, L.st[1].col_of,
                          L.st[2].col_of, L.st[3].col_of};
      J.lamL = L.st[1].lam_out;
      J.fL1 = L.fL1;
      J.fL2 = L.fL2;
      J.fR1 = L.fR1;
      J.fR2 = L.fR2;
      J.sigma_out = u.sigma_out;
      J.signs = L.signs;
      J.defl = u.defl;
      for (int k = 0; k < 4; ++k) {
        J.flags[k] = L.st[k].flags;
        J.fN[k] = L.st[k].N;
      }
      if (u.defl) P.any_defl = true;
      bn[i] = cdiv(u.n, 256);
      for (int k = 0; k < 4; ++k) P.host_stages.push_back(L.st[k]);
    }
    const std::vector<int> off = prefix(bn);
    P.prob.n = nu;
    P.prob.blocks_n = off.back();
    P.prob.boff_n = B.put(off);
    P.prob.job = B.put(jobs);
    P.prob.counters = counters;
    P.prob.ncounters = counters ? 2 * kNumShapes : 0;
  }
  // projections: U^T a and V^T [b w1 w2]
  {
    std::vector<GemvJob> jobs;
    for (const Update& u : ups) {
      const Layout& L = u.L;
      GemvJob ju{u.m, u.m, u.ldu, 1, gemv_cblocks(u.m), gemv_chunks(u.m), u.U, {u.a, nullptr, nullptr},
                 {L.p, nullptr, nullptr}, L.gemv_pu};
      GemvJob jv{u.n, u.n, u.ldv, 3, gemv_cblocks(u.n), gemv_chunks(u.n), u.V, {u.b, L.w1, L.w2},
                 {L.q, L.t1, L.t2}, L.gemv_pv};
      jobs.push_back(jv);
      jobs.push_back(ju);
    }
    std::vector<int> bp, br;
    for (const GemvJob& j : jobs) {
      bp.push_back(j.cblocks * j.chunks);
      br.push_back(cdiv(j.nv * j.N, 256));
    }
    const std::vector<int> op = prefix(bp), orr = prefix(br);
    P.gemv.n = (int)jobs.size();
    P.gemv.blocks_p = op.back();
    P.gemv.blocks_r = orr.back();
    P.gemv.boff_p = B.put(op);
    P.gemv.boff_r = B.put(orr);
    P.gemv.job = B.put(jobs);
  }
  // eigen-update levels, largest first
  for (int lev = 0; lev < 2; ++lev) {
    std::vector<Stage> st;
    std::vector<TmvJob> tv;
    for (const Update& u : ups) {
      const Layout& L = u.L;
      if (lev == 0) {
        st.push_back(L.st[0]);
        tv.push_back(TmvJob{3, {L.yLm, L.pL1, L.pL2}, {L.zLm, L.pL1b, L.pL2b}});
        st.push_back(L.st[2]);
        tv.push_back(TmvJob{3, {L.yRm, L.t1, L.t2}, {L.zRm, L.pR1b, L.pR2b}});
      } else {
        st.push_back(L.st[1]);
        tv.push_back(TmvJob{2, {L.pL1b, L.pL2b, nullptr}, {L.fL1, L.fL2, nullptr}});
        st.push_back(L.st[3]);
        tv.push_back(TmvJob{2, {L.pR1b, L.pR2b, nullptr}, {L.fR1, L.fR2, nullptr}});
      }
    }
    P.lev[lev] = build_level(st, tv, B);
  }
  // products, grouped by tile shape, largest first within a group (FP64 and
  // split FP32), or the slicing and slice products of the INT8 form
  P.slices = opt.slices;
  for (int lev = 0; lev < 2 && precision == SVDU_PREC_SLICED_INT8; ++lev) {
    std::vector<SliceXJob> xs;
    std::vector<SliceCJob> cs;
    std::vector<I8Job> gs;
    for (const Update& u : ups) {
      const Layout& L = u.L;
      for (int side = 0; side < 2; ++side) {
        const int N = side == 0 ? u.m : u.n;
        const double* X = lev == 0 ? (side == 0 ? u.U : u.V) : (side == 0 ? L.TL : L.TR);
        const int ldx = lev == 0 ? (side == 0 ? u.ldu : u.ldv) : N;
        double* Xo = lev == 0 ? (side == 0 ? L.TL : L.TR) : (side == 0 ? u.U_out : u.V_out);
        const int ldo = lev == 0 ? N : (side == 0 ? u.ldu_out : u.ldv_out);
        CauchyDesc d = desc_of(L.st[2 * side + lev], (lev == 1 && side == 1) ? L.signs : nullptr);
        if (side == 1 && u.n > u.m) d = with_members(d, L.st[2 * side + lev]);
        const int KB = i8_pad(N, kI8K) / kI8K, Rp = i8_pad(N, kI8BM), Cp = i8_pad(N, kI8BN);
        xs.push_back(SliceXJob{N, N, ldx, KB, Rp / 16, X, L.i8A[side], L.i8ea[side], L.status});
        cs.push_back(SliceCJob{d, KB, Cp / 16, L.i8B[side], L.i8eb[side]});
        gs.push_back(I8Job{N, N, ldo, KB, Rp / kI8BM, Cp / kI8BN, (Rp / kI8BM) * (Cp / kI8BN), L.i8A[side],
                           L.i8B[side], L.i8ea[side], L.i8eb[side], Xo, X, ldx, d});
      }
    }
    std::vector<int> bx, bc, bg;
    for (const SliceXJob& j : xs) bx.push_back(j.rblocks);
    for (const SliceCJob& j : cs) bc.push_back(j.cblocks);
    for (const I8Job& j : gs) bg.push_back(j.tiles);
    const std::vector<int> ox = prefix(bx), oc = prefix(bc), og = prefix(bg);
    P.sx[lev] = SliceXList{(int)xs.size(), ox.back(), B.put(ox), B.put(xs)};
    P.sc[lev] = SliceCList{(int)cs.size(), oc.back(), B.put(oc), B.put(cs)};
    P.i8[lev] = I8List{(int)gs.size(), og.back(), B.put(og), B.put(gs)};
  }
  for (int lev = 0; lev < 2 && precision != SVDU_PREC_SLICED_INT8; ++lev) {
    std::vector<GemmJob> by_shape[kNumShapes];
    for (const Update& u : ups) {
      const Layout& L = u.L;
      GemmJob g[2];
      if (lev == 0) {
        g[0] = make_gemm_job(u.m, u.U, u.ldu, desc_of(L.st[0]), L.TL, u.m, precision, opt);
        const CauchyDesc dr = desc_of(L.st[2]);
        g[1] = make_gemm_job(u.n, u.V, u.ldv, u.n > u.m ? with_members(dr, L.st[2]) : dr, L.TR, u.n, precision,
                             opt);
      } else {
        g[0] = make_gemm_job(u.m, L.TL, u.m, desc_of(L.st[1]), u.U_out, u.ldu_out, precision, opt);
        const CauchyDesc dr = desc_of(L.st[3], L.signs);
        g[1] = make_gemm_job(u.n, L.TR, u.n, u.n > u.m ? with_members(dr, L.st[3]) : dr, u.V_out, u.ldv_out,
                             precision, opt);
      }
      for (int k = 0; k < 2; ++k) by_shape[g[k].shape].push_back(g[k]);
    }
    for (int sh = 0; sh < kNumShapes; ++sh)
      P.gemm[lev][sh] = build_gemm_list(by_shape[sh], counters ? counters + lev * kNumShapes + sh : nullptr, B);
  }
  // column renormalisation of the precision form
  {
    std::vector<RenormJob> jobs;
    if (precision == SVDU_PREC_SPLIT32) {
      for (const Update& u : ups) {
        jobs.push_back(RenormJob{u.n, u.n, u.ldv_out, cdiv(u.n, 256), cdiv(u.n, 128), u.V_out, u.L.renorm_v,
                                 u.L.status});
        jobs.push_back(RenormJob{u.m, u.m, u.ldu_out, cdiv(u.m, 256), cdiv(u.m, 128), u.U_out, u.L.renorm_u,
                                 u.L.status});
      }
    }
    std::vector<int> bl;
    for (const RenormJob& j : jobs) bl.push_back(j.cblocks * j.chunks);
    const std::vector<int> o = prefix(bl);
    P.renorm.n = (int)jobs.size();
    P.renorm.blocks = o.back();
    P.renorm.boff = B.put(o);
    P.renorm.job = B.put(jobs);
  }
  // refinement of close clusters (FP64 only)
  {
    std::vector<RefineJob> jobs;
    std::vector<int> bn, bc, bw, bcl;
    if (precision != SVDU_PREC_SPLIT32) {
      for (const Update& u : ups) {
        const Layout& L = u.L;
        RefineJob R{};
        R.m = u.m;
        R.n = u.n;
        R.kmax = L.kmax;
        R.cmax = L.cmax;
        R.U = u.U;
        R.V = u.V;
        R.a = u.a;
        R.b = u.b;
        R.sigma = u.sigma;
        R.ldu = u.ldu;
        R.ldv = u.ldv;
        R.Uo = u.U_out;
        R.so = u.sigma_out;
        R.Vo = u.V_out;
        R.lduo = u.ldu_out;
        R.ldvo = u.ldv_out;
        R.status = L.status;
        R.info = L.rf_info;
        R.cl_start = L.rf_start;
        R.cl_size = L.rf_size;
        R.cl_off = L.rf_off;
        R.col_idx = L.rf_idx;
        R.Yu = L.rf_Yu;
        R.Yv = L.rf_Yv;
        R.T = L.rf_T;
        R.W = L.rf_W;
        R.beta = L.rf_beta;
        jobs.push_back(R);
        bn.push_back(cdiv(u.n, 256));
        bc.push_back(cdiv(u.m + 1, 16));   // refine_vt_kernel: 16 columns of [V b] per block
        bw.push_back(cdiv(u.m, 4));
        bcl.push_back(std::min(32, L.cmax));
      }
    }
    const std::vector<int> on = prefix(bn), oc = prefix(bc), ow = prefix(bw), ocl = prefix(bcl);
    RefineList& F = P.refine;
    F.n = (int)jobs.size();
    F.blocks_n = on.back();
    F.blocks_c = oc.back();
    F.blocks_w = ow.back();
    F.blocks_cl = ocl.back();
    F.boff_n = B.put(on);
    F.boff_c = B.put(oc);
    F.boff_w = B.put(ow);
    F.boff_cl = B.put(ocl);
    F.job = B.put(jobs);
  }
  blob->resize((blob->size() + 15) & ~size_t(15));
}

// ---------------------------------------------------------------------------
// blob upload through kernel arguments
// ---------------------------------------------------------------------------
constexpr int kChunkWords = 120;   // 1920 bytes per launch
struct BlobChunk {
  int words;
  uint4 data[kChunkWords];
};

__global__ void write_blob_kernel(BlobChunk c, uint4* dst) {
  for (int i = threadIdx.x; i < c.words; i += blockDim.x) dst[i] = c.data[i];
}

void write_blob(const std::vector<char>& blob, char* dst, hipStream_t st) {
  const size_t words = blob.size() / 16;
  for (size_t w0 = 0; w0 < words; w0 += kChunkWords) {
    BlobChunk c;
    c.words = (int)std::min<size_t>(kChunkWords, words - w0);
    memcpy(c.data, blob.data() + w0 * 16, (size_t)c.words * 16);
    hipLaunchKernelGGL(write_blob_kernel, dim3(1), dim3(128), 0, st, c, reinterpret_cast<uint4*>(dst) + w0);
  }
}

// ---------------------------------------------------------------------------
// the sequence
// ---------------------------------------------------------------------------
void enqueue_plan(const Plan& P, const Sched& S, int part, hipStream_t st,
                  const std::function<void(int)>* after_level) {
  const bool s32 = P.precision == SVDU_PREC_SPLIT32;
  if (part != kStepProductsOnward) {
    S.mark(0, st);
    if (P.prob.blocks_n > 0)
      hipLaunchKernelGGL(prob_init_kernel, dim3(P.prob.blocks_n), dim3(256), 0, st, P.prob);
    launch_gemv_list(P.gemv, st);
    S.mark(1, st);
    if (P.prob.n > 0) hipLaunchKernelGGL(prob_setup_kernel, dim3(P.prob.n), dim3(1024), 0, st, P.prob);
    for (int lev = 0; lev < 2; ++lev) {
      launch_stage_level(P.lev[lev], S.maxit, S.secular_ff, st);
      launch_cauchy_tmatvec_level(P.lev[lev], st);
      if (after_level) (*after_level)(lev);
    }
    if (P.prob.blocks_n > 0)
      hipLaunchKernelGGL(prob_finalize_kernel, dim3(P.prob.blocks_n), dim3(256), 0, st, P.prob);
    S.mark(2, st);
  }
  if (part == kStepUpToRoots) return;
  if (part == kStepAll) {
    for (int lev = 0; lev < 2; ++lev) {
      if (P.precision == SVDU_PREC_SLICED_INT8) {
        launch_slice_x(P.sx[lev], P.slices, st);
        launch_slice_c(P.sc[lev], P.slices, st);
        launch_gemm_i8(P.i8[lev], P.slices, st);
        S.mark(3 + lev, st);
        continue;
      }
      for (int sh = 0; sh < kNumShapes; ++sh) {
        const GemmList& G = P.gemm[lev][sh];
        const int cap = S.grid_cap[s32 ? 1 : 0][sh];
        const bool pers = S.persistent && G.counter && cap > 0;
        if (s32)
          launch_gemm_split32(G, sh, pers, cap, st);
        else
          launch_gemm_f64(G, sh, pers, cap, st);
      }
      if (lev == 1 && s32) launch_column_renorm(P.renorm, st);
      S.mark(3 + lev, st);
    }
  }
  if (S.refine) launch_refine(P.refine, st);
  if (P.any_defl && P.prob.blocks_n > 0)
    hipLaunchKernelGGL(prob_flags_kernel, dim3(P.prob.blocks_n), dim3(256), 0, st, P.prob);
  S.mark(5, st);
}

void enqueue_status_gather(const Plan& P, int* out, hipStream_t st) {
  if (P.prob.n <= 0) return;
  hipLaunchKernelGGL(prob_status_kernel, dim3((P.prob.n + 255) / 256), dim3(256), 0, st, P.prob, out);
}

// ---------------------------------------------------------------------------
// tile shapes: a table per precision and size bucket in every context, filled
// by the autotuner (svdu_autotune); the defaults are what it measured on
// MI355X.
// ---------------------------------------------------------------------------
void default_shape_table(int (&t)[kNumPrec][kShapeBuckets]) {
  static const int def[kNumPrec][kShapeBuckets] = {
      {kT64x64, kT128x128, kT128x64, kT128x64, kT128x128, kT256x128k64, kT256x128k64, kT256x128k64},
      {kT64x64, kT64x64, kT64x64, kT64x64, kT64x64, kT64x128, kT128x128, kT128x128}};
  memcpy(t, def, sizeof(def));
}

int shape_bucket(int N) {
  int b = 0;
  int lim = 64;
  while (b < kShapeBuckets - 1 && N > lim) {
    ++b;
    lim *= 2;
  }
  return b;
}

int choose_shape(int N, int precision, const Options& o) {
  if (o.forced_shape >= 0) return o.forced_shape;
  return o.shape_table[precision == SVDU_PREC_SPLIT32 ? 1 : 0][shape_bucket(N)];
}

int gemm_f64_grid_cap(int shape);
int gemm_split32_grid_cap(int shape);
int gemm_grid_cap(int shape, int precision) {
  return precision == SVDU_PREC_SPLIT32 ? gemm_split32_grid_cap(shape) : gemm_f64_grid_cap(shape);
}

}  // namespace svdu

svdu_ctx::~svdu_ctx() {
  // the pinned memory may still be read by the last call's plan upload
  if (upload_pending && uploaded) (void)hipEventSynchronize(uploaded);
  for (hipStream_t s : {aux, aux2})
    if (s) (void)hipStreamDestroy(s);   // work already enqueued on it still completes
  for (hipEvent_t e : {fork, join, roots[0], roots[1], up0, done_a, done_b, uploaded})
    if (e) (void)hipEventDestroy(e);
  if (pinned) (void)hipHostFree(pinned);
}

namespace svdu {

// ---------------------------------------------------------------------------
// timing ring of a context
// ---------------------------------------------------------------------------
TimingRing::~TimingRing() {
  for (int c = 0; c < kRingCalls; ++c)
    if (made[c])
      for (int k = 0; k < kRingEvents; ++k) (void)hipEventDestroy(ev[c][k]);
}

int TimingRing::begin() {
  if (!on || count >= kRingCalls) return -1;
  const int c = count;
  if (!made[c]) {
    for (int k = 0; k < kRingEvents; ++k)
      if (hipEventCreate(&ev[c][k]) != hipSuccess) {
        for (int j = 0; j < k; ++j) (void)hipEventDestroy(ev[c][j]);
        return -1;
      }
    made[c] = true;
  }
  ++count;
  return c;
}

void TimingRing::mark(int call, int k, hipStream_t st) {
  if (call >= 0) (void)hipEventRecord(ev[call][k], st);
}

int TimingRing::set(bool v) {
  const int old = on ? 1 : 0;
  on = v;
  count = 0;
  return old;
}

int TimingRing::read(double* ms, int max_calls) {
  const int n = std::min(count, max_calls);
  for (int c = 0; c < n; ++c) {
    if (hipEventSynchronize(ev[c][kRingEvents - 1]) != hipSuccess) return SVDU_EHIP;
    for (int k = 0; k + 1 < kRingEvents; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[c][k], ev[c][k + 1]) != hipSuccess) return SVDU_EHIP;
      ms[c * (kRingEvents - 1) + k] = t;
    }
  }
  return n;
}

Sched sched_of(svdu_ctx* ctx, const Options& o, bool persistent, bool timed) {
  Sched S;
  S.maxit = o.maxit;
  S.secular_ff = o.secular_ff;
  S.refine = o.refine;
  S.persistent = persistent;
  if (ctx && persistent && !ctx->have_caps) {
    for (int p = 0; p < kNumPrec; ++p)
      for (int s = 0; s < kNumShapes; ++s) ctx->grid_cap[p][s] = gemm_grid_cap(s, p);
    ctx->have_caps = true;
  }
  if (ctx && ctx->have_caps) memcpy(S.grid_cap, ctx->grid_cap, sizeof(S.grid_cap));
  if (ctx && timed) {
    S.tcall = ctx->ring.begin();
    S.ring = S.tcall >= 0 ? &ctx->ring : nullptr;
  }
  return S;
}

int status_code(int h) {
  if (h & kStNonFinite) return SVDU_ENONFINITE;
  if (h & kStBadSigma) return SVDU_EBADSIGMA;
  if (h & kStNoConv) return SVDU_ENOCONV;
  return SVDU_OK;
}

}  // namespace svdu
