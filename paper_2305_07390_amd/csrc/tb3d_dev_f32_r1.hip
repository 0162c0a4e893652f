// Compiled variants of the device-tiled 3D pass: f32, radius 1.
#include "tb3d_dev_impl.hpp"

namespace stencil_impl {
template hipError_t tb3d_dev_launch_r<float, 1>(int, int, const Tb3dDevParams<float>*, hipStream_t);
}  // namespace stencil_impl
