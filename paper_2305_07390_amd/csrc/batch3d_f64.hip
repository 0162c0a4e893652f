// Persistent batch kernels, 3D, f64: every (radius, pattern) at its deepest depth.
#include "batch_impl.hpp"

namespace stencil_impl {
hipError_t tb3d_batch_launch_f64(int r, int shape, const void* params, int grid, hipStream_t s) {
  const auto* p = (const Batch3DParams<double>*)params;
  switch (r) {
    case 1: return batch::launch3d_shape<double, 1>(shape, p, grid, s);
    case 2: return batch::launch3d_shape<double, 2>(shape, p, grid, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace stencil_impl
