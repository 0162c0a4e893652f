// The fused persistent batch kernel, f64.
#include "batch_impl.hpp"

namespace stencil_impl {
hipError_t batch_launch_f64(const void* params, int grid, size_t lds, hipStream_t s) {
  return batch::launch<double, 0>((const BatchParams<double>*)params, grid, lds, s);
}
hipError_t batch_launch_f64_aux(const void* params, int grid, size_t lds, hipStream_t s) {
  return batch::launch<double, 1>((const BatchParams<double>*)params, grid, lds, s);
}
}  // namespace stencil_impl
