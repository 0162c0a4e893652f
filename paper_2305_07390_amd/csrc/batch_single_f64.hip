// Single-variant persistent kernels, f64 (one per variant with a blocked
// single-grid kernel; see batch_impl.hpp).
#include "batch_impl.hpp"

namespace stencil_impl {
hipError_t batch_launch_single_f64(int variant, const void* params, int grid, size_t lds, hipStream_t s) {
  return batch::launch_single_from<double, 0>(variant, (const BatchParams<double>*)params, grid, lds, s);
}
}  // namespace stencil_impl
