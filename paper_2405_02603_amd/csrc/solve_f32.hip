// Single-precision instantiation of the solve passes.
#include "solve_launch.hpp"

namespace fsp {
hipError_t solve_f32(const SolveGeom& g, const void* rho, void* phi, int first, int last, hipStream_t s) {
  return launch_solve<float>(g, rho, phi, first, last, s);
}
}  // namespace fsp
