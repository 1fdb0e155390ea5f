// Device helpers shared by the svdu kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svdu {

constexpr double kU = 1.1102230246251565e-16;  // unit roundoff 2^-53

// 1/x to within an ulp for |x| >= 2^-1000: hardware reciprocal (about 2^-24
// relative) refined by two Newton steps.
__device__ __forceinline__ double recip_fast(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
// Below this |x| recip_fast is not used (1 / x may overflow there).
__device__ __forceinline__ bool recip_tiny(double x) { return __builtin_fabs(x) < 0x1p-1000; }
// num / x: num times recip_fast(x) where that applies, a true division below
// (where 1 / x alone can overflow although num / x does not).
__device__ __forceinline__ double div_by(double num, double x) {
  return recip_tiny(x) ? num / x : num * recip_fast(x);
}

// Global-memory access through a generic pointer. Pointers read from job
// tables are generic to the compiler; casting them to the global address space
// gives global (not flat) loads and stores, which the memory counters track
// apart from LDS traffic.
template <class T>
__device__ __forceinline__ T gld(const T* p) {
  return *((const __attribute__((address_space(1))) T*)p);
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
  *((__attribute__((address_space(1))) T*)p) = v;
}
// 16-byte load of two consecutive doubles (p 16-byte aligned).
__device__ __forceinline__ double2 gld2(const double* p) {
  typedef double dv2 __attribute__((ext_vector_type(2)));
  const dv2 v = *((const __attribute__((address_space(1))) dv2*)p);
  return double2{v.x, v.y};
}

// Butterfly reductions over a full wave of 64 lanes. IEEE addition and
// multiplication commute, so every lane ends with the same bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// The same over aligned groups of G lanes (G a power of two, at most 64):
// every lane of a group ends with the same bits, and G = 64 is the whole wave
// in the same order as wave_sum.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <int G>
__device__ __forceinline__ double group_prod(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v *= __shfl_xor(v, o, 64);
  return v;
}
template <int G>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = __builtin_fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <int G>
__device__ __forceinline__ bool group_any(bool b) {
  int x = b ? 1 : 0;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x != 0;
}

// Block-wide inclusive scan of one int per thread (blockDim a multiple of 64,
// at most 4096). `sh` holds at least 64 ints of shared memory. Returns the
// inclusive prefix; *total receives the block total.
__device__ inline int block_scan_incl(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) sh[w] = v;
  __syncthreads();
  if (w == 0) {
    int s = (lane < nw) ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int t = __shfl_up(s, o, 64);
      if (lane >= o) s += t;
    }
    if (lane < nw) sh[lane] = s;
  }
  __syncthreads();
  if (w > 0) v += sh[w - 1];
  *total = sh[nw - 1];
  __syncthreads();
  return v;
}

// Block-wide sum of one double per thread; every thread gets the result.
__device__ inline double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += sh[k];  // fixed order: deterministic
  __syncthreads();
  return s;
}

// Counter-based hash to a double in [-1, 1) (splitmix64 finaliser).
__device__ __forceinline__ double hash_unit(uint64_t i, uint64_t stream) {
  uint64_t x = i * 0x9E3779B97F4A7C15ull + stream * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull;
  x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27; x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * 0x1p-52 - 1.0;
}

}  // namespace svdu
