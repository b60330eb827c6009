// Double-precision instantiation of the solve passes.
#include "solve_launch.hpp"

namespace fsp {
hipError_t solve_f64(const SolveGeom& g, const void* rho, void* phi, int first, int last, hipStream_t s) {
  return launch_solve<double>(g, rho, phi, first, last, s);
}
}  // namespace fsp
