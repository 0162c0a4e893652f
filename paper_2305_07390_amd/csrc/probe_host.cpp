// Host side of the microbenchmarks (probe.hip): buffers, launches and timing.
// Every probe allocates its own device memory on the caller's stream, times
// its kernels with events on that stream, synchronises it and releases the
// memory before returning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "launch.hpp"
#include "plan.hpp"

namespace stencil_impl {
hipError_t probe_copy_launch(const void* src, void* dst, int64_t bytes, int grid, int variant, hipStream_t s);
hipError_t probe_chain_init_launch(uint32_t* buf, uint32_t n, uint32_t stride, uint32_t a, hipStream_t s);
hipError_t probe_chase_hbm_launch(const uint32_t* buf, uint32_t stride, int steps, uint32_t* out, hipStream_t s);
hipError_t probe_chase_lds_launch(int steps, uint32_t a, uint32_t* out, hipStream_t s);
hipError_t probe_chain_fma_launch(int steps, double a, double b, double* out, hipStream_t s);
hipError_t probe_lds_bw_launch(int grid, int iters, uint32_t* out, hipStream_t s);
hipError_t probe_neighbor_sync_launch(int mode, double* buf, unsigned* flags, unsigned* err,
                                      unsigned long long* mismatches, int gx, int gy, int rounds, int words,
                                      long long timeout, hipStream_t s);
}  // namespace stencil_impl

using namespace stencil_impl;

namespace {

// Events around `launch` on s; seconds of the bracketed work.
template <typename F>
stencil_status time_on(hipStream_t s, F launch, double* seconds) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "probe");
  *seconds = ms * 1e-3;
  return STENCIL_OK;
}

constexpr uint32_t kLcgA = 0x9E3779B1u;  // = 1 mod 4: a full-period walk mod 2^k

}  // namespace

extern "C" {

stencil_status stencil_probe_copy(int64_t bytes, void* stream, double* bytes_per_s) {
  if (!bytes_per_s || bytes < ((int64_t)1 << 20) || bytes > ((int64_t)64 << 30))
    return fail(STENCIL_ERR_INVALID, "bytes in [1 MiB, 64 GiB] and a result pointer");
  *bytes_per_s = 0;
  bytes = bytes / 4096 * 4096;
  hipStream_t s = (hipStream_t)stream;
  DeviceInfo di = device_info();
  if (!di.ok) return fail(STENCIL_ERR_DEVICE, "no device");
  char* buf = nullptr;
  hipError_t e = hipMallocAsync((void**)&buf, (size_t)2 * bytes, s);
  if (e != hipSuccess) return fail(STENCIL_ERR_NOMEM, "copy probe: %s", hipGetErrorString(e));
  stencil_status st = STENCIL_OK;
  e = hipMemsetAsync(buf, 1, (size_t)bytes, s);
  if (e != hipSuccess) st = hip_fail(e, "copy probe fill");
  // kernel variants x grids of 4 .. 32 workgroups per CU; each timed three
  // times after a warm-up run, the best time over all
  double best = 1e30;
  for (int variant = 0; variant < 4 && st == STENCIL_OK; ++variant) {
    for (int per_cu = 4; per_cu <= 32 && st == STENCIL_OK; per_cu *= 2) {
      const int grid = di.cus * per_cu;
      for (int rep = 0; rep < 4 && st == STENCIL_OK; ++rep) {
        double t = 0;
        st = time_on(s, [&] { return probe_copy_launch(buf, buf + bytes, bytes, grid, variant, s); }, &t);
        if (rep > 0) best = std::min(best, t);
      }
    }
  }
  (void)hipFreeAsync(buf, s);
  (void)hipStreamSynchronize(s);
  if (st == STENCIL_OK) *bytes_per_s = 2.0 * (double)bytes / best;
  return st;
}

stencil_status stencil_probe_latency(int32_t kind, void* stream, double* seconds) {
  if (!seconds) return fail(STENCIL_ERR_INVALID, "NULL result");
  *seconds = 0;
  hipStream_t s = (hipStream_t)stream;
  uint32_t* buf = nullptr;
  stencil_status st = STENCIL_OK;
  hipError_t e;
  if (kind == STENCIL_PROBE_HBM_LATENCY) {
    // 2^22 links 256 bytes apart: a 1 GiB footprint, four times the
    // last-level cache
    const uint32_t n = 1u << 22, stride = 64;
    e = hipMallocAsync((void**)&buf, (size_t)n * stride * 4 + 256, s);
    if (e != hipSuccess) return fail(STENCIL_ERR_NOMEM, "latency probe: %s", hipGetErrorString(e));
    uint32_t* out = buf + (size_t)n * stride;
    e = probe_chain_init_launch(buf, n, stride, kLcgA, s);
    if (e != hipSuccess) st = hip_fail(e, "latency probe init");
    double t1 = 0, t2 = 0;
    const int a = 20000, b = 120000;
    if (st == STENCIL_OK) st = time_on(s, [&] { return probe_chase_hbm_launch(buf, stride, a, out, s); }, &t1);
    if (st == STENCIL_OK) st = time_on(s, [&] { return probe_chase_hbm_launch(buf, stride, b, out, s); }, &t2);
    if (st == STENCIL_OK) *seconds = (t2 - t1) / (double)(b - a);  // launch cost cancels
    (void)hipFreeAsync(buf, s);
    (void)hipStreamSynchronize(s);
    return st;
  }
  if (kind == STENCIL_PROBE_LDS_LATENCY || kind == STENCIL_PROBE_FMA64_LATENCY) {
    e = hipMallocAsync((void**)&buf, 256, s);
    if (e != hipSuccess) return fail(STENCIL_ERR_NOMEM, "latency probe: %s", hipGetErrorString(e));
    double t1 = 0, t2 = 0;
    const int a = 1 << 18, b = 1 << 22;
    auto run = [&](int steps) {
      return kind == STENCIL_PROBE_LDS_LATENCY ? probe_chase_lds_launch(steps, kLcgA, buf, s)
                                               : probe_chain_fma_launch(steps, 1.0000001, 1e-9, (double*)buf, s);
    };
    st = time_on(s, [&] { return run(a); }, &t1);
    if (st == STENCIL_OK) st = time_on(s, [&] { return run(b); }, &t2);
    if (st == STENCIL_OK) *seconds = (t2 - t1) / (double)(b - a);
    (void)hipFreeAsync(buf, s);
    (void)hipStreamSynchronize(s);
    return st;
  }
  return fail(STENCIL_ERR_INVALID, "unknown latency probe %d", kind);
}

stencil_status stencil_probe_lds_bandwidth(void* stream, double* bytes_per_s) {
  if (!bytes_per_s) return fail(STENCIL_ERR_INVALID, "NULL result");
  *bytes_per_s = 0;
  hipStream_t s = (hipStream_t)stream;
  DeviceInfo di = device_info();
  if (!di.ok) return fail(STENCIL_ERR_DEVICE, "no device");
  uint32_t* out = nullptr;
  hipError_t e = hipMallocAsync((void**)&out, 256, s);
  if (e != hipSuccess) return fail(STENCIL_ERR_NOMEM, "LDS probe: %s", hipGetErrorString(e));
  const int grid = 2 * di.cus;  // two workgroups (eight waves) per CU
  double t1 = 0, t2 = 0;
  const int a = 2000, b = 40000;
  stencil_status st = time_on(s, [&] { return probe_lds_bw_launch(grid, a, out, s); }, &t1);
  if (st == STENCIL_OK) st = time_on(s, [&] { return probe_lds_bw_launch(grid, b, out, s); }, &t2);
  // bytes read per workgroup and iteration: 8 x 256 lanes x 16 bytes
  if (st == STENCIL_OK) *bytes_per_s = (double)grid * (double)(b - a) * 8 * 256 * 16 / (t2 - t1);
  (void)hipFreeAsync(out, s);
  (void)hipStreamSynchronize(s);
  return st;
}

stencil_status stencil_probe_neighbor_sync(int32_t mode, int32_t rounds, int32_t payload_bytes, void* stream,
                                           double* seconds_per_round, uint64_t* mismatches) {
  if (!seconds_per_round || !mismatches || rounds < 1 || rounds > 1000000 || payload_bytes < 0 ||
      payload_bytes > (1 << 20) || (mode != 0 && mode != 1))
    return fail(STENCIL_ERR_INVALID, "mode 0/1, rounds in [1, 1e6], payload in [0, 1 MiB], result pointers");
  *seconds_per_round = 0;
  *mismatches = 0;
  hipStream_t s = (hipStream_t)stream;
  DeviceInfo di = device_info();
  if (!di.ok) return fail(STENCIL_ERR_DEVICE, "no device");
  // the most square torus of one workgroup per CU
  int gx = 1;
  for (int f = 1; f * f <= di.cus; ++f)
    if (di.cus % f == 0) gx = f;
  const int gy = di.cus / gx;
  const int words = payload_bytes / 8;
  const size_t buf_bytes = (size_t)di.cus * 2 * words * 8;
  const size_t ctl = 4096 + (size_t)di.cus * 4;
  char* mem = nullptr;
  hipError_t e = hipMallocAsync((void**)&mem, ctl + buf_bytes + 256, s);
  if (e != hipSuccess) return fail(STENCIL_ERR_NOMEM, "neighbour probe: %s", hipGetErrorString(e));
  unsigned* err = (unsigned*)mem;
  unsigned long long* bad = (unsigned long long*)(mem + 256);
  unsigned* flags = (unsigned*)(mem + 4096);
  double* buf = (double*)(mem + (ctl + 255) / 256 * 256);
  stencil_status st = STENCIL_OK;
  const long long timeout = 500000000;  // 5 s of the 100 MHz clock
  double t = 0;
  for (int rep = 0; rep < 2 && st == STENCIL_OK; ++rep) {
    e = hipMemsetAsync(mem, 0, ctl + buf_bytes, s);
    if (e != hipSuccess) {
      st = hip_fail(e, "neighbour probe reset");
      break;
    }
    const int r = rep == 0 ? std::min(rounds, 64) : rounds;
    st = time_on(s, [&] {
      return probe_neighbor_sync_launch(mode, buf, flags, err, bad, gx, gy, r, words, timeout, s);
    }, &t);
  }
  unsigned herr = 0;
  unsigned long long hbad = 0;
  if (st == STENCIL_OK) {
    e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "neighbour probe read-back");
  }
  (void)hipFreeAsync(mem, s);
  (void)hipStreamSynchronize(s);
  if (st != STENCIL_OK) return st;
  if (herr) return fail(STENCIL_ERR_TIMEOUT, "a neighbour wait expired");
  *seconds_per_round = t / rounds;
  *mismatches = hbad;
  return STENCIL_OK;
}

}  // extern "C"
