// Compiled variants of the blocked 2D pass: f64, radius 3.
#include "tb2d_impl.hpp"

namespace stencil_impl {
template hipError_t tb2d_launch_r<double, 3>(int, int, const Tb2dParams<double>*, int, int, size_t,
                                            hipStream_t);
}  // namespace stencil_impl
