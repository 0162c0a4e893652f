// stencil_run_noalloc: the one-shot run for callers that cannot allocate
// device memory (code under stream capture, tight serving loops). It plans
// like stencil_run, but the ping-pong workspace of a multi-pass plan is a
// fixed region of library-owned device memory instead of a stream-ordered
// allocation, and the call makes no device allocation or release of any kind.
//
// The region is a file-scope device array. Host code never uses its name as
// an address (that would be a host-side stand-in); the device address comes
// from hipGetSymbolAddress, taken once per device with that device current
// and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)STENCIL_NOALLOC_SCRATCH_BYTES;

// Every GPU that runs this entry point holds its own copy until the process
// ends. Its contents are whatever the last call left; every pass writes the
// cells it later reads (the halo frame is copied in first), so nothing has to
// start at zero.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];
bool g_done[kMaxDevices];
hipError_t g_err[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first
// call per device).
stencil_status scratch_address(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return stencil_impl::hip_fail(e, "no-alloc run: current device");
  if (dev < 0 || dev >= kMaxDevices)
    return stencil_impl::fail(STENCIL_ERR_DEVICE, "no-alloc run: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_done[dev]) {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = p;
    g_done[dev] = true;
  }
  if (g_err[dev] != hipSuccess) return stencil_impl::hip_fail(g_err[dev], "no-alloc run: scratch address");
  if (!g_ptr[dev]) return stencil_impl::fail(STENCIL_ERR_DEVICE, "no-alloc run: scratch address is NULL");
  *ptr = g_ptr[dev];
  return STENCIL_OK;
}

}  // namespace

extern "C" {

stencil_status stencil_run_noalloc(const double* coeffs, int32_t radius, const stencil_shape* shape,
                                   stencil_dtype dtype, int64_t T, const void* in, void* out, void* stream) {
  if (!in || !out) return stencil_impl::fail(STENCIL_ERR_INVALID, "in/out is NULL");
  stencil_plan_t plan = nullptr;
  // overlapped tiles only: a device-tiled plan reports bounded-wait expiries
  // through a per-stream word that is allocated on a stream's first use
  stencil_tuning hint;
  hint.tile[0] = hint.tile[1] = hint.tile[2] = 0;
  hint.depth = 0;
  hint.flags = STENCIL_FLAG_OVERLAPPED_TILING;
  stencil_status st = stencil_plan(&plan, coeffs, radius, shape, dtype, T, &hint);
  if (st != STENCIL_OK) return st;
  const size_t wbytes = plan->workspace;
  if (wbytes > kScratchBytes) {
    stencil_plan_destroy(plan);
    return stencil_impl::fail(STENCIL_ERR_INVALID,
                              "no-alloc run: the plan needs %zu bytes of workspace, more than the %zu-byte "
                              "scratch region (use stencil_run or stencil_execute)",
                              wbytes, kScratchBytes);
  }
  void* ws = nullptr;
  if (wbytes > 0) st = scratch_address(&ws);
  if (st == STENCIL_OK) st = stencil_execute(plan, in, out, ws, stream);
  stencil_plan_destroy(plan);
  return st;
}

}  // extern "C"
