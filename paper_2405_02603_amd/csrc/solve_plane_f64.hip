// Plane-kernel launchers (double): passes 1-2 and 4-5 fused per i0-plane, every supported size.
#include "solve_launch.hpp"

namespace fsp {
template hipError_t launch_plane<double>(int, int, bool, const PlaneArgs&, int, hipStream_t);
}  // namespace fsp
