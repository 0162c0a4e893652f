// Single-variant persistent kernels, f32 (one per variant with a blocked
// single-grid kernel; see batch_impl.hpp).
#include "batch_impl.hpp"

namespace stencil_impl {
hipError_t batch_launch_single_f32(int variant, const void* params, int grid, size_t lds, hipStream_t s) {
  return batch::launch_single_from<float, 0>(variant, (const BatchParams<float>*)params, grid, lds, s);
}
}  // namespace stencil_impl
