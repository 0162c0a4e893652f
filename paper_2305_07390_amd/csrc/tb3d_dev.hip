// Dispatch of the device-tiled 3D pass to its compiled variants, and the
// small helpers its host side needs.
#include "tb3d_dev_impl.hpp"

namespace stencil_impl {

#define TB3D_DEV_EXTERN(T, R) \
  extern template hipError_t tb3d_dev_launch_r<T, R>(int, int, const Tb3dDevParams<T>*, hipStream_t);
TB3D_DEV_EXTERN(double, 1)
TB3D_DEV_EXTERN(double, 2)
TB3D_DEV_EXTERN(float, 1)
TB3D_DEV_EXTERN(float, 2)
#undef TB3D_DEV_EXTERN

hipError_t tb3d_dev_launch(int dtype, int r, int shape, int cdepth, const void* params, hipStream_t stream) {
  if (cdepth < 1 || cdepth > tb3dd::dev_max_depth_c(dtype, r, shape)) return hipErrorInvalidValue;
  if (dtype == kF64) {
    const auto* p = (const Tb3dDevParams<double>*)params;
    if (r == 1) return tb3d_dev_launch_r<double, 1>(shape, cdepth, p, stream);
    if (r == 2) return tb3d_dev_launch_r<double, 2>(shape, cdepth, p, stream);
  } else if (dtype == kF32) {
    const auto* p = (const Tb3dDevParams<float>*)params;
    if (r == 1) return tb3d_dev_launch_r<float, 1>(shape, cdepth, p, stream);
    if (r == 2) return tb3d_dev_launch_r<float, 2>(shape, cdepth, p, stream);
  }
  return hipErrorInvalidValue;
}

int tb3d_dev_max_depth(int dtype, int r, int shape) {
  if (r < 1 || r > 2 || shape < kStar || shape > kGeneral) return 0;
  return tb3dd::dev_max_depth_c(dtype, r, shape);
}

int tb3d_dev_tile_y() { return tb3d::LY; }

int64_t tb3d_dev_ring_elems(int r, int cdepth) {
  return r == 1 ? tb3dd::ring_per_tile<1, 1>(cdepth) : tb3dd::ring_per_tile<2, 1>(cdepth);
}

int64_t tb3d_dev_iterations(int r, int d, int64_t Qz) { return Qz + r + (int64_t)(d - 1) * (r + tb3dd::lag_of(r)); }

namespace {
__global__ __launch_bounds__(256) void fill_zero_u32_kernel(unsigned int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
}  // namespace

hipError_t fill_zero_u32_launch(unsigned int* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace stencil_impl
