// An entry point that allocates nothing: gpuqt_moments with its workspace in a
// fixed device array of this library instead of a caller buffer, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

// Workspace of gpuqt_moments_noalloc.  Every GPU the library runs on holds its
// own copy until the process ends.  In host code the name stands for a
// host-side symbol, not the device address: the address comes from
// hipGetSymbolAddress, per device, and only that address is used.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
gpuqt_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return gpuqt::set_error(GPUQT_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return gpuqt::set_error(GPUQT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GPUQT_OK;
}

}  // namespace

size_t gpuqt_noalloc_scratch_bytes(void) { return kScratchBytes; }

gpuqt_status gpuqt_moments_noalloc(gpuqt_h h, int32_t B, const double* phiL, const double* phiR, int32_t M,
                                   double* mu, void* stream) {
  if (!h) return gpuqt::set_error(GPUQT_ERR_ARG, "NULL handle");
  if (M < 0) return gpuqt::set_error(GPUQT_ERR_ARG, "M must be >= 0");
  size_t need = 0;
  gpuqt_status st = gpuqt_workspace_size(h, GPUQT_OP_MOMENTS, B, M, 0, &need);
  if (st) return st;
  if (need > kScratchBytes)
    return gpuqt::set_error(GPUQT_ERR_WORKSPACE,
                            "gpuqt_moments_noalloc needs " + std::to_string(need) +
                                " bytes of workspace for this n, B and M; its fixed array holds " +
                                std::to_string(kScratchBytes) + " (use gpuqt_moments with a workspace)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return gpuqt::set_error(GPUQT_ERR_HIP, "hipGetDevice failed");
  void* ws = nullptr;
  if ((st = scratch_address(dev, &ws))) return st;
  return gpuqt_moments(h, B, phiL, phiR, M, mu, ws, kScratchBytes, stream);
}
