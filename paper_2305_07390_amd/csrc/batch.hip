// Batch dispatch and the batched halo-frame copy.
#include "device_common.hpp"
#include "launch.hpp"
#include "batch_impl.hpp"

namespace stencil_impl {

hipError_t batch_launch_f64(const void* params, int grid, size_t lds, hipStream_t s);
hipError_t batch_launch_f64_aux(const void* params, int grid, size_t lds, hipStream_t s);
hipError_t batch_launch_f32(const void* params, int grid, size_t lds, hipStream_t s);

hipError_t batch_launch(int dtype, const void* params, int grid, size_t lds_bytes, hipStream_t stream,
                        bool aux) {
  if (aux) return dtype == kF64 ? batch_launch_f64_aux(params, grid, lds_bytes, stream) : hipErrorInvalidValue;
  if (dtype == kF64) return batch_launch_f64(params, grid, lds_bytes, stream);
  if (dtype == kF32) return batch_launch_f32(params, grid, lds_bytes, stream);
  return hipErrorInvalidValue;
}

int batch_max_depth(int dtype, int ndim, int r, int shape) {
  if (r < 1 || r > kMaxR || shape < kStar || shape > kGeneral) return 0;
  if (ndim == 3 && r > 2) return 0;
  if (ndim != 2 && ndim != 3) return 0;
  return batch::batch_depth_c(dtype, ndim, r, shape);
}

hipError_t batch_launch_single_f64(int variant, const void* params, int grid, size_t lds, hipStream_t s);
hipError_t batch_launch_single_f32(int variant, const void* params, int grid, size_t lds, hipStream_t s);

hipError_t batch_launch_single(int dtype, int variant, const void* params, int grid, size_t lds_bytes,
                               hipStream_t stream) {
  if (dtype == kF64) return batch_launch_single_f64(variant, params, grid, lds_bytes, stream);
  if (dtype == kF32) return batch_launch_single_f32(variant, params, grid, lds_bytes, stream);
  return hipErrorInvalidValue;
}

bool batch_single_supported(int dtype, int ndim, int r, int shape) {
  if (shape < kStar || shape > kGeneral || (ndim != 2 && ndim != 3)) return false;
  return batch::single_supported(dtype, ndim, r, shape);
}

int batch_single_depth(int dtype, int ndim, int r, int shape) {
  return batch_single_supported(dtype, ndim, r, shape) ? batch::single_depth_c(dtype, ndim, r, shape) : 0;
}

int batch_aux_depth(int dtype, int ndim, int r, int shape) {
  if (r < 1 || r > kMaxR || shape < kStar || shape > kGeneral) return 0;
  return batch::aux_depth_c(dtype, ndim, r, shape);
}

namespace {
template <typename Real, int R>
size_t lds_3d(int shape) {
  using namespace tb3d;
  switch (shape) {
    case kStar: return Lds<Real, R, cells_y(sizeof(Real) == 8, R, kStar)>::kBytes;
    case kBox: return Lds<Real, R, cells_y(sizeof(Real) == 8, R, kBox)>::kBytes;
    default: return Lds<Real, R, cells_y(sizeof(Real) == 8, R, kGeneral)>::kBytes;
  }
}
}  // namespace

size_t batch_lds_3d(int dtype, int r, int shape) {
  const bool f64 = dtype == kF64;
  if (r == 1) return f64 ? lds_3d<double, 1>(shape) : lds_3d<float, 1>(shape);
  if (r == 2) return f64 ? lds_3d<double, 2>(shape) : lds_3d<float, 2>(shape);
  return 0;
}

namespace {

// Grid-wide synchronisation probe: `rounds` device-wide barriers of the whole
// grid (one workgroup per CU) through one counter in device memory, the
// mechanism that separates passes in the persistent launches. Every wait is
// bounded by the realtime-clock watchdog; an expired wait sets *err and the
// workgroup leaves.
__global__ __launch_bounds__(64) void grid_sync_probe_kernel(unsigned int* ctr, unsigned int* err,
                                                             int rounds, long long timeout_ticks) {
  const int lane = (int)threadIdx.x;
  const unsigned g = gridDim.x;
  for (int k = 0; k < rounds; ++k) {
    __hip_atomic_fetch_add(ctr, lane == 0 ? 1u : 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned need = (unsigned)(k + 1) * g;
    const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
    bool ok = true;
    while (true) {
      const unsigned v = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
      if (v >= need) break;
      if ((long long)__builtin_amdgcn_s_memrealtime() - t0 > timeout_ticks) {
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ok) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
}

// Fold a launch's own error word into a report word read by stencil_sync.
__global__ __launch_bounds__(64) void error_fold_kernel(const unsigned int* src, unsigned int* dst) {
  if (threadIdx.x == 0) {
    const unsigned v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v != 0u) __hip_atomic_fetch_or(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// blockIdx.y = job, blockIdx.x strides over the padded rows (z, y) of that job.
template <typename Real>
__global__ __launch_bounds__(64) void frame_copy_batch_kernel(const FrameCopyJob* __restrict__ jobs) {
  const FrameCopyJob& J = jobs[blockIdx.y];
  const Real* __restrict__ src = (const Real*)J.src;
  Real* __restrict__ dst = (Real*)J.dst;
  const int64_t e0 = J.ext[0], e1 = J.ext[1], e2 = J.ext[2];
  const int r0 = J.r[0], r1 = J.r[1], r2 = J.r[2];
  const int64_t nrows = e0 * e1;
  for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int64_t z = row / e1, y = row - z * e1;
    const bool halo_row = z < r0 || z >= e0 - r0 || y < r1 || y >= e1 - r1;
    const int64_t base = row * e2;
    if (halo_row) {
      for (int64_t x = threadIdx.x; x < e2; x += blockDim.x) dst[base + x] = src[base + x];
    } else {
      for (int64_t k = threadIdx.x; k < 2 * r2; k += blockDim.x) {
        const int64_t x = k < r2 ? k : e2 - 2 * r2 + k;
        dst[base + x] = src[base + x];
      }
    }
  }
}

}  // namespace

hipError_t grid_sync_probe_launch(unsigned int* ctr, unsigned int* err, int rounds, int grid,
                                  long long timeout_ticks, hipStream_t stream) {
  hipLaunchKernelGGL(grid_sync_probe_kernel, dim3(grid), dim3(64), 0, stream, ctr, err, rounds,
                     timeout_ticks);
  return hipGetLastError();
}

hipError_t error_fold_launch(const unsigned int* src, unsigned int* dst, hipStream_t stream) {
  hipLaunchKernelGGL(error_fold_kernel, dim3(1), dim3(64), 0, stream, src, dst);
  return hipGetLastError();
}

hipError_t frame_copy_batch_launch(int dtype, const FrameCopyJob* jobs_dev, int njobs,
                                   hipStream_t stream) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(2048, (unsigned)njobs);
  if (dtype == kF64) {
    hipLaunchKernelGGL(frame_copy_batch_kernel<double>, grid, dim3(64), 0, stream, jobs_dev);
  } else if (dtype == kF32) {
    hipLaunchKernelGGL(frame_copy_batch_kernel<float>, grid, dim3(64), 0, stream, jobs_dev);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace stencil_impl
