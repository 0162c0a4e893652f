// Compiled variants of the blocked 3D pass: f32, radius 2.
#include "tb3d_impl.hpp"

namespace stencil_impl {
template hipError_t tb3d_launch_r<float, 2>(int, int, const Tb3dParams<float>*, int, hipStream_t);
}  // namespace stencil_impl
