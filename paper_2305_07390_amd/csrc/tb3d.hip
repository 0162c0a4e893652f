// Dispatch of the temporally blocked 3D pass to its compiled variants.
#include "tb3d_impl.hpp"

namespace stencil_impl {

#define TB3D_EXTERN(T, R) \
  extern template hipError_t tb3d_launch_r<T, R>(int, int, const Tb3dParams<T>*, int, hipStream_t);
TB3D_EXTERN(double, 1)
TB3D_EXTERN(double, 2)
TB3D_EXTERN(float, 1)
TB3D_EXTERN(float, 2)
#undef TB3D_EXTERN

hipError_t tb3d_launch(int dtype, int r, int shape, int depth, const void* params, int grid,
                       hipStream_t stream) {
  if (depth < 1 || depth > tb3d::max_depth_c(dtype, r, shape)) return hipErrorInvalidValue;
  if (dtype == kF64) {
    const auto* p = (const Tb3dParams<double>*)params;
    if (r == 1) return tb3d_launch_r<double, 1>(shape, depth, p, grid, stream);
    if (r == 2) return tb3d_launch_r<double, 2>(shape, depth, p, grid, stream);
  } else if (dtype == kF32) {
    const auto* p = (const Tb3dParams<float>*)params;
    if (r == 1) return tb3d_launch_r<float, 1>(shape, depth, p, grid, stream);
    if (r == 2) return tb3d_launch_r<float, 2>(shape, depth, p, grid, stream);
  }
  return hipErrorInvalidValue;
}

int tb3d_cells_y(int dtype, int r, int shape) { return tb3d::cells_y(dtype == kF64, r, shape); }

int tb3d_max_depth(int dtype, int r, int shape) {
  (void)dtype;
  if (r < 1 || r > 2 || shape < kStar || shape > kGeneral) return 0;
  return tb3d::max_depth_c(dtype, r, shape);
}

}  // namespace stencil_impl
