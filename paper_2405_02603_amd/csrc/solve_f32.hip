// float solve driver: passes of a launch group, and the tile of the axis-0 pass.
#define FSP_SPLIT_LAUNCHERS
#include "solve_launch.hpp"

namespace fsp {
hipError_t solve_f32(const SolveGeom& g, int first, int last, hipStream_t s) {
  return launch_solve<float>(g, first, last, s);
}

// Column tile of the axis-0 pass for pencil length L (the Green's octant is stored in such tiles).
int conv_tile_f32(int L) { return col_tiles<float>(L); }
}  // namespace fsp
