// Internal interfaces of libsvdu: per-stage device buffers and kernel launchers.
//
// One symmetric rank-one eigen-update (the paper's RankOneUpdate, Section 6.2)
// is a "stage". Its input is a basis X whose columns carry eigenvalues lam_in
// (storage order), the projected vector z = X^T v and rho. Its output is the
// description of the orthogonal matrix C~ (equation CTildeFinalForm1) as
// per-row and per-output-column data, from which every kernel that needs an
// entry of C~ regenerates it:
//
//   live column c (a secular root mu_c = d_org + tau):
//     C~[j, c] = zeta_j * s_c / ((rg_j - o_c) - tau_c)      (0 where zeta_j == 0)
//   deflated column c (a kept pole, member `mem` of cluster `cl`):
//     C~[j, c] = (rcl_j == cl) ? ([j == mem] - 2 rh_j h_c) : 0
//
// where rg_j is the (merged) pole of row j, zeta_j its Loewner weight with the
// sign of z_j, s_c = 1/|c_c| the column scale, and rh the Householder vector
// of an exactly repeated pole group (zero for single poles and dropped rows).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace svdu {

enum StatusBits : int {
  kStNoConv = 1,      // a secular root hit the iteration cap
  kStNonFinite = 2,   // NaN or Inf in an input (or produced from one)
  kStBadSigma = 4,    // sigma / eigenvalues not in the required order, or negative sigma
};
// Once a fatal bit is set every later kernel of the call returns at entry, so
// no index is ever derived from invalid data.
constexpr int kStFatal = kStNonFinite | kStBadSigma;

struct Stage {
  int N = 0;              // dimension of the eigenproblem
  int* status = nullptr;  // device status word of the call
  int cap = 0;            // allocated length of every per-index array
  double* rho = nullptr;  // device scalar
  bool descending = false;  // output columns by descending eigenvalue
  // inputs
  const double* lam_in = nullptr;  // N, storage order of X's columns
  int* col_of = nullptr;           // N, sorted position -> storage column
  double* z = nullptr;             // N, storage order
  // deflation (sorted positions t)
  double* dsort = nullptr;
  double* zs = nullptr;
  int* clu = nullptr;      // cluster id, -1 for a dropped component
  int* Llist = nullptr;    // sorted positions of kept components
  double* g = nullptr;     // per cluster: pole
  double* W = nullptr;     // per cluster: norm of z over the cluster
  double* W2 = nullptr;    // per cluster: W^2
  int* cfirst = nullptr;   // per cluster: first index into Llist
  int* csize = nullptr;    // per cluster: member count
  int* dlist = nullptr;    // deflated sorted positions (dropped or non-first member)
  double* dval = nullptr;  // their eigenvalues
  int* counts = nullptr;   // [0] K clusters (= roots), [1] Kd deflated, [2] kept count
  // roots and weights (per cluster / root index)
  int* org = nullptr;
  double* tau = nullptr;
  double* mu = nullptr;
  double* what = nullptr;
  double* cs = nullptr;    // 1 / column norm
  int* iters = nullptr;    // secular iterations per root
  // row descriptors (storage order)
  double* rg = nullptr;
  double* rzeta = nullptr;
  double* rh = nullptr;
  int* rcl = nullptr;
  int8_t* flags = nullptr;  // 0 kept, 1 dropped (zero component), 2 merged repeated pole
  // column descriptors (output position)
  int8_t* ctype = nullptr;  // 0 live, 1 deflated
  double* co = nullptr;
  double* ctau = nullptr;
  double* ccs = nullptr;
  int* ccl = nullptr;
  int* cmem = nullptr;
  double* ch = nullptr;
  double* lam_out = nullptr;  // eigenvalue per output column
  int* rootpos = nullptr;     // output position of each root
  int* dpos = nullptr;        // output position of each deflated item
  double* hx = nullptr;       // per cluster x 3: Householder dot products for C~^T x
};

// Descriptor view handed to the product kernels.
struct CauchyDesc {
  int N;
  const double* rg;
  const double* rzeta;
  const double* rh;
  const int* rcl;
  const int8_t* ctype;
  const double* co;
  const double* ctau;
  const double* ccs;
  const int* ccl;
  const int* cmem;
  const double* ch;
  const double* colscale;  // optional per-output-column sign (nullptr: none)
  const int* status;       // device status word; fatal bits make the kernels return
  // cluster members (with_members): the FP64 product then writes whole
  // 64-column chunks of deflated columns as copies and one reflection.
  // nullptr: those columns are generated like any other.
  const int* counts;   // [0] number of clusters
  const int* cfirst;   // per cluster: first index into Llist
  const int* csize;    // per cluster: member count
  const int* Llist;    // sorted positions of kept components
  const int* col_of;   // sorted position -> row of C~
};

__host__ __device__ inline CauchyDesc desc_of(const Stage& s, const double* colscale = nullptr) {
  return CauchyDesc{s.N, s.rg, s.rzeta, s.rh, s.rcl, s.ctype, s.co, s.ctau, s.ccs, s.ccl, s.cmem, s.ch,
                    colscale, s.status, nullptr, nullptr, nullptr, nullptr, nullptr};
}

// For products that can hold whole chunks of deflated columns (the zero block
// of the right-hand products when n > m).
__host__ __device__ inline CauchyDesc with_members(CauchyDesc d, const Stage& s) {
  d.counts = s.counts;
  d.cfirst = s.cfirst;
  d.csize = s.csize;
  d.Llist = s.Llist;
  d.col_of = s.col_of;
  return d;
}

// Launchers over job lists are declared in jobs.h.

// FMM path of the product (k_fmm.hip). The plan of a product is built on the
// host from host copies of the stage's K poles and roots, all plans of a call
// are uploaded in one copy, then the kernels are enqueued.
struct FmmPrepared;
size_t fmm_workspace_elems(int R, int N);
size_t fmm_plan_bytes(int N);

}  // namespace svdu
