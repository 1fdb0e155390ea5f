// svdu_rank1_update_noalloc: the direct-path rank-1 update without a caller
// workspace, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The update's workspace is a file-scope device array (`scratch`, one copy per
// device, held until the process ends). Host code never uses the array's name
// as an address: on the first call on a device (with that device current) the
// device address is looked up with hipGetSymbolAddress and kept per device,
// and only that address is handed to the kernels. The launch sequence is the
// one of svdu_rank1_update, so the results are bitwise the same. Every call on
// a device shares its array: calls that overlap on one device race (the
// sequence's first kernel resets the status word and tile counters; every
// other workspace entry is written before it is read).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/svdu.h"
#include "engine.h"

namespace {

constexpr size_t kScratchBytes = SVDU_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` per device (nullptr: not looked up yet)

// The address of this device's array, looked up once per device.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return SVDU_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SVDU_EHIP;
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return SVDU_OK;
}

// The call's status code (SVDU_OK or a negative SVDU_E* code) from the status
// bits of the update's workspace.
__global__ void export_status(const int* bits, int* out) {
  if (threadIdx.x == 0) {
    const int h = *bits;
    *out = (h & svdu::kStNonFinite) ? SVDU_ENONFINITE
         : (h & svdu::kStBadSigma)  ? SVDU_EBADSIGMA
         : (h & svdu::kStNoConv)    ? SVDU_ENOCONV
                                    : SVDU_OK;
  }
}

}  // namespace

extern "C" int svdu_rank1_update_noalloc(svdu_ctx* ctx, int m, int n, const double* U, int ldu, const double* sigma,
                                         const double* V, int ldv, const double* a, const double* b, int precision,
                                         double* U_out, int ldu_out, double* sigma_out, double* V_out, int ldv_out,
                                         int8_t* defl, int* status, void* stream) {
  if (!ctx) return SVDU_EINVAL;
  if (m < 1 || n < m) return SVDU_EINVAL;
  if (precision != SVDU_PREC_FP64 && precision != SVDU_PREC_SPLIT32) return SVDU_EINVAL;
  const size_t need = svdu_workspace_bytes(m, n, SVDU_PATH_DIRECT, precision);
  if (need == 0) return SVDU_EINVAL;
  if (need > kScratchBytes) return SVDU_ENOMEM;
  if (const int rc = svdu::ctx_device_check(ctx)) return rc;
  void* ws = nullptr;
  if (const int rc = scratch_address(ctx->device, &ws)) return rc;
  const int rc = svdu_rank1_update(ctx, m, n, U, ldu, sigma, V, ldv, a, b, 0.0, SVDU_PATH_DIRECT, precision, U_out,
                                   ldu_out, sigma_out, V_out, ldv_out, defl, ws, kScratchBytes, stream);
  if (rc != SVDU_OK) return rc;
  if (status) {
    hipLaunchKernelGGL(export_status, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       static_cast<const int*>(ws), status);
    if (hipGetLastError() != hipSuccess) return SVDU_EHIP;
  }
  return SVDU_OK;
}
