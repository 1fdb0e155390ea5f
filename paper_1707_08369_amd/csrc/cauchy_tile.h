// Cauchy tile generation shared by the kernels that need entries of C~
// (see svdu_internal.h for the descriptor layout).
#pragma once
#include "device_util.h"
#include "svdu_internal.h"

namespace svdu {

typedef double d4 __attribute__((ext_vector_type(4)));

// K step of the product kernels.
constexpr int kBK = 16;

// Entry C~[j, c] from the descriptors (see svdu_internal.h).
struct ColDesc {
  int type;   // -1 out of range, 0 live, 1 deflated
  double o, t, s, h;
  int cl, mem;
};

__device__ __forceinline__ ColDesc load_col(const CauchyDesc& d, int c) {
  ColDesc r{-1, 0.0, 0.0, 0.0, 0.0, -1, -1};
  if (c < d.N) {
    r.type = gld(d.ctype + c);
    r.o = gld(d.co + c);
    r.t = gld(d.ctau + c);
    r.s = gld(d.ccs + c);
    r.h = gld(d.ch + c);
    r.cl = gld(d.ccl + c);
    r.mem = gld(d.cmem + c);
  }
  return r;
}

// Column descriptor for the product kernels. Columns past N become live
// columns with scale 0 and a shift far from every pole: their entries are
// zeros from the branch-free path (and are never stored), so a ragged last
// column tile keeps its block on that path.
__device__ __forceinline__ ColDesc load_col_tile(const CauchyDesc& d, int c) {
  if (c < d.N) return load_col(d, c);
  return ColDesc{0, 0.0, -0x1p1000, 0.0, 0.0, -1, -1};
}

struct RowVals {
  double z, g, h;
  int cl;
};

__device__ __forceinline__ double live_entry(double z, double g, const ColDesc& c, double* absd) {
  const double del = (g - c.o) - c.t;
  *absd = __builtin_fabs(del);
  double r = __builtin_amdgcn_rcp(del);
  double e = __builtin_fma(-del, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-del, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double v = (z * c.s) * r;
  return (z == 0.0) ? 0.0 : v;
}

// For a live column this is the value live_entry computes (the same refined
// reciprocal), so an entry does not depend on which path generated it.
__device__ __forceinline__ double general_entry(int j, const RowVals& rv, const ColDesc& c) {
  if (c.type == 0) {
    if (rv.z == 0.0) return 0.0;
    return div_by(rv.z * c.s, (rv.g - c.o) - c.t);
  }
  if (c.type < 0 || rv.cl != c.cl) return 0.0;
  return ((j == c.mem) ? 1.0 : 0.0) - 2.0 * rv.h * c.h;
}

template <bool LIVE>
__device__ __forceinline__ double gen_entry(const CauchyDesc& d, int j, int N, const ColDesc& c, double* mind) {
  const int jj = j < N ? j : N - 1;
  const double zl = gld(d.rzeta + jj);   // unconditional load (index clamped), then select
  const double z = (j < N) ? zl : 0.0;
  const double g = gld(d.rg + jj);
  if (LIVE) {
    double ad;
    const double v = live_entry(z, g, c, &ad);
    *mind = __builtin_fmin(*mind, ad);
    return v;
  } else {
    RowVals rv{z, g, gld(d.rh + jj), (j < N) ? gld(d.rcl + jj) : -2};
    return general_entry(j, rv, c);
  }
}


// Tile shapes of the product kernels: W waves stacked along M, each wave
// 16 MB rows (MB = 1 or 2 MFMA blocks of 16) by 64 NC columns (NC = 1 or 2).
// kT128x128k32: 128 x 128 with LDS tiles of 32 k rows, one barrier per 32 k.
// kT256x128k64: 8 waves of 32 x 128 (256 x 128), LDS tiles of 64 k rows
// (one barrier per 64 k); every generated C~ entry serves 256 rows of X.
enum TileShape : int {
  kT128x128 = 0, kT64x128 = 1, kT128x64 = 2, kT64x64 = 3, kT128x128k32 = 4, kT256x128k64 = 5, kNumShapes = 6
};
__host__ __device__ constexpr int shape_bm(int s) {
  return (s == kT64x128 || s == kT64x64) ? 64 : (s == kT256x128k64 ? 256 : 128);
}
__host__ __device__ constexpr int shape_bn(int s) { return (s == kT128x64 || s == kT64x64) ? 64 : 128; }
// The shape a product actually runs with. The split-FP32 kernel has no
// staged or 8-wave variant and runs those shapes as 128 x 128.
__host__ __device__ constexpr int run_shape(int s, bool split32) {
  return (split32 && s >= kT128x128k32) ? kT128x128 : s;
}

// XCD-aware order of a job's 2-D tile grid. Consecutive blocks of a launch
// are dealt to the 8 XCDs in turn, so local tiles t with equal t % 8 share an
// XCD whatever the job's first block is; they are given consecutive tiles of
// one block row (sharing an X panel, and that XCD's L2).
__device__ __forceinline__ void tile_origin(int t, int tiles, int tiles_n, int bm, int bn, int* m0, int* n0) {
  const int full = (tiles / 8) * 8;
  const int lid = (t < full) ? (t % 8) * (tiles / 8) + t / 8 : t;
  *m0 = (lid / tiles_n) * bm;
  *n0 = (lid % tiles_n) * bn;
}

}  // namespace svdu
