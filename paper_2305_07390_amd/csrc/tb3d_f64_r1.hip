// Compiled variants of the blocked 3D pass: f64, radius 1.
#include "tb3d_impl.hpp"

namespace stencil_impl {
template hipError_t tb3d_launch_r<double, 1>(int, int, const Tb3dParams<double>*, int, hipStream_t);
}  // namespace stencil_impl
