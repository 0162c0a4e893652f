// Persistent batch kernels, 2D, f64: every (radius, pattern) at its deepest depth.
#include "batch_impl.hpp"

namespace stencil_impl {
hipError_t tb2d_batch_launch_f64(int r, int shape, const void* params, int grid, size_t lds,
                                  hipStream_t s) {
  const auto* p = (const Batch2DParams<double>*)params;
  switch (r) {
    case 1: return batch::launch2d_shape<double, 1>(shape, p, grid, lds, s);
    case 2: return batch::launch2d_shape<double, 2>(shape, p, grid, lds, s);
    case 3: return batch::launch2d_shape<double, 3>(shape, p, grid, lds, s);
    case 4: return batch::launch2d_shape<double, 4>(shape, p, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace stencil_impl
