// Compiled variants of the device-tiled 3D pass: f64, radius 2.
#include "tb3d_dev_impl.hpp"

namespace stencil_impl {
template hipError_t tb3d_dev_launch_r<double, 2>(int, int, const Tb3dDevParams<double>*, hipStream_t);
}  // namespace stencil_impl
