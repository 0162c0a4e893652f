// Batch dispatch and the batched halo-frame copy.
#include "device_common.hpp"
#include "launch.hpp"

namespace stencil_impl {

hipError_t tb2d_batch_launch_f64(int r, int shape, const void* params, int grid, size_t lds, hipStream_t s);
hipError_t tb2d_batch_launch_f32(int r, int shape, const void* params, int grid, size_t lds, hipStream_t s);
hipError_t tb3d_batch_launch_f64(int r, int shape, const void* params, int grid, hipStream_t s);
hipError_t tb3d_batch_launch_f32(int r, int shape, const void* params, int grid, hipStream_t s);

hipError_t tb2d_batch_launch(int dtype, int r, int shape, int depth, const void* params, int grid,
                             size_t lds_bytes, hipStream_t stream) {
  (void)depth;  // each job carries its depths; the kernel holds the deepest
  if (dtype == kF64) return tb2d_batch_launch_f64(r, shape, params, grid, lds_bytes, stream);
  if (dtype == kF32) return tb2d_batch_launch_f32(r, shape, params, grid, lds_bytes, stream);
  return hipErrorInvalidValue;
}

hipError_t tb3d_batch_launch(int dtype, int r, int shape, int depth, const void* params, int grid,
                             hipStream_t stream) {
  (void)depth;
  if (dtype == kF64) return tb3d_batch_launch_f64(r, shape, params, grid, stream);
  if (dtype == kF32) return tb3d_batch_launch_f32(r, shape, params, grid, stream);
  return hipErrorInvalidValue;
}

namespace {

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
