// Compiled variants of the blocked 2D pass: f32, radius 3.
#include "tb2d_impl.hpp"

namespace stencil_impl {
template hipError_t tb2d_launch_r<float, 3>(int, int, const Tb2dParams<float>*, int, int, size_t,
                                            hipStream_t);
}  // namespace stencil_impl
