// The fused persistent batch kernel, f32.
#include "batch_impl.hpp"

namespace stencil_impl {
hipError_t batch_launch_f32(const void* params, int grid, size_t lds, hipStream_t s) {
  return batch::launch<float, 0>((const BatchParams<float>*)params, grid, lds, s);
}
}  // namespace stencil_impl
