// Plain one-step kernel (no temporal blocking): one thread per interior cell,
// terms in dense-box order with one fused multiply-add each (paper Section 2.1,
// Listings 1-3). It serves radius 0, radii or patterns without a blocked
// variant, and as the t = 1 streaming baseline. The caller copies the halo into
// the destination once; this kernel writes interior cells only.
#include "device_common.hpp"
#include "launch.hpp"

namespace stencil_impl {
using namespace stencil_dev;

namespace {

template <typename Real>
__global__ __launch_bounds__(256) void naive_kernel(const NaiveParams<Real> p) {
  const Real* __restrict__ src = (const Real*)p.src;
  Real* __restrict__ dst = (Real*)p.dst;
  const int64_t nx = p.hi[2] - p.lo[2];
  const int64_t ny = p.hi[1] - p.lo[1];
  const int64_t nz = p.hi[0] - p.lo[0];
  const int64_t total = nx * ny * nz;
  const int ntaps = p.ntaps;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = c % nx;
    const int64_t t = c / nx;
    const int64_t y = t % ny;
    const int64_t z = t / ny;
    const int64_t i = ((z + p.lo[0]) * p.ext[1] + (y + p.lo[1])) * p.ext[2] + x + p.lo[2];
    Real acc = Real(0);
    for (int q = 0; q < ntaps; ++q) acc = fma_t(p.w[q], src[i + p.off[q]], acc);
    dst[i] = acc;
  }
}

// Copy every halo cell (a cell with some coordinate within r of the padded
// array's edge) from src to dst. One block per padded row (z, y); a halo row is
// copied whole, any other row only its first and last r cells.
template <typename Real>
__global__ __launch_bounds__(256) void frame_copy_kernel(const Real* __restrict__ src,
                                                         Real* __restrict__ dst, int64_t e0,
                                                         int64_t e1, int64_t e2, int r0, int r1,
                                                         int r2) {
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

hipError_t frame_copy_launch(int dtype, const void* src, void* dst, const int64_t ext[3],
                             const int r[3], hipStream_t stream) {
  int64_t rows = ext[0] * ext[1];
  int64_t blocks = rows < 65536 ? rows : 65536;
  if (blocks < 1) blocks = 1;
  if (dtype == kF64) {
    hipLaunchKernelGGL(frame_copy_kernel<double>, dim3((unsigned)blocks), dim3(64), 0, stream,
                       (const double*)src, (double*)dst, ext[0], ext[1], ext[2], r[0], r[1], r[2]);
  } else if (dtype == kF32) {
    hipLaunchKernelGGL(frame_copy_kernel<float>, dim3((unsigned)blocks), dim3(64), 0, stream,
                       (const float*)src, (float*)dst, ext[0], ext[1], ext[2], r[0], r[1], r[2]);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t naive_launch(int dtype, const void* params, int64_t cells, hipStream_t stream) {
  int64_t blocks = (cells + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  void* args[] = {(void*)params};
  if (dtype == kF64)
    return hipLaunchKernel((const void*)&naive_kernel<double>, dim3((unsigned)blocks), dim3(256),
                           args, 0, stream);
  if (dtype == kF32)
    return hipLaunchKernel((const void*)&naive_kernel<float>, dim3((unsigned)blocks), dim3(256),
                           args, 0, stream);
  return hipErrorInvalidValue;
}

}  // namespace stencil_impl
