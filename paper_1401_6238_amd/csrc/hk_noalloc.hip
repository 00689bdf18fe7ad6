// hankel_tvp_noalloc: the equal-vector product of hankel_tvp (Section 3
// procedures with x_1 = ... = x_m = x) with its workspace in a static device
// array instead of a caller-provided buffer, for callers that cannot allocate
// device memory.
//
// `scratch` below is a device-side array: in host code its name is only a
// host stand-in, so every host use goes through the device address that
// hipGetSymbolAddress returns for the current device (one copy of the array
// per device, each at its own address).  The address is looked up once per
// device, on that device's first call, and kept for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/hankel.h"
#include "hk_plan.hpp"

namespace hk {
// Records the thread-local error of a failed call (hk_api.cpp).
hk_status_t api_finish(const Status &s);
}  // namespace hk

// The workspace of every hankel_tvp_noalloc call on a device.  Nothing in it
// needs to start at zero: the column pass writes every workspace column the
// row pass reads (pruned columns are never read), and the row pass writes
// every partial sum the reduction reads, so the previous call's contents are
// harmless.
static __device__ __align__(256) unsigned char scratch[HK_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES];  // device address of `scratch` per device; nullptr until looked up
}  // namespace

// Device address of `scratch` on the current device (looked up on first use).
static hk::Status scratch_on_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hk::fail(HK_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES)
    return hk::fail(HK_ERR_DEVICE, "device index " + std::to_string(dev) + " is beyond the " +
                                       std::to_string(MAX_DEVICES) + " devices hankel_tvp_noalloc supports");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hk::fail(HK_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (!p) return hk::fail(HK_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hk::Status();
}

extern "C" hk_status_t hankel_tvp_noalloc(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x, void *y,
                                          void *alpha, hipStream_t stream) {
  // shape checks and the workspace this product needs (host only)
  size_t need = 0;
  const hk_status_t rc = hankel_tvp_workspace_size(dt, m, n, &need);
  if (rc != HK_SUCCESS) return rc;
  if (need > HK_NOALLOC_SCRATCH_BYTES)
    return hk::api_finish(hk::fail(
        HK_ERR_WORKSPACE, "this product needs " + std::to_string(need) + " bytes of workspace; hankel_tvp_noalloc "
                          "holds at most HK_NOALLOC_SCRATCH_BYTES = " + std::to_string((size_t)HK_NOALLOC_SCRATCH_BYTES) +
                          " (use hankel_tvp with a caller-provided workspace)"));
  void *ws = nullptr;
  const hk::Status s = scratch_on_current_device(&ws);
  if (!s.ok()) return hk::api_finish(s);
  // the existing entry point, with the static array as its workspace
  return hankel_tvp(dt, h, m, n, x, y, alpha, ws, HK_NOALLOC_SCRATCH_BYTES, stream);
}
