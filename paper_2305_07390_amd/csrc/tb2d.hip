// Dispatch of the temporally blocked 2D pass to its compiled variants.
#include "tb2d_impl.hpp"

namespace stencil_impl {

#define TB2D_EXTERN(T, R)                                                                     \
  extern template hipError_t tb2d_launch_r<T, R>(int, int, const Tb2dParams<T>*, int, int,   \
                                                 size_t, hipStream_t);
TB2D_EXTERN(double, 1)
TB2D_EXTERN(double, 2)
TB2D_EXTERN(double, 3)
TB2D_EXTERN(double, 4)
TB2D_EXTERN(float, 1)
TB2D_EXTERN(float, 2)
TB2D_EXTERN(float, 3)
TB2D_EXTERN(float, 4)
#undef TB2D_EXTERN

namespace {
template <typename Real>
hipError_t launch_r(int r, int shape, int depth, const Tb2dParams<Real>* p, int grid, int block,
                    size_t lds, hipStream_t s) {
  switch (r) {
    case 1: return tb2d_launch_r<Real, 1>(shape, depth, p, grid, block, lds, s);
    case 2: return tb2d_launch_r<Real, 2>(shape, depth, p, grid, block, lds, s);
    case 3: return tb2d_launch_r<Real, 3>(shape, depth, p, grid, block, lds, s);
    case 4: return tb2d_launch_r<Real, 4>(shape, depth, p, grid, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t tb2d_launch(int dtype, int r, int shape, int depth, const void* params, int grid,
                       int block, size_t lds_bytes, hipStream_t stream) {
  if (depth < 1 || depth > max_depth_c(dtype == kF64, r, shape)) return hipErrorInvalidValue;
  if (dtype == kF64)
    return launch_r<double>(r, shape, depth, (const Tb2dParams<double>*)params, grid, block,
                            lds_bytes, stream);
  if (dtype == kF32)
    return launch_r<float>(r, shape, depth, (const Tb2dParams<float>*)params, grid, block,
                           lds_bytes, stream);
  return hipErrorInvalidValue;
}

int tb2d_max_depth(int dtype, int r, int shape) {
  if (r < 1 || r > kMaxR || shape < kStar || shape > kGeneral) return 0;
  return max_depth_c(dtype == kF64, r, shape);
}

int tb2d_cols_per_lane(int dtype, int r, int shape) { return tb2d_cols(dtype == kF64, r, shape); }

}  // namespace stencil_impl
