// Column-pass launchers (double): every length and schedule variant of P2, P3 and P4.
#include "solve_launch.hpp"

namespace fsp {
template hipError_t launch_col<double>(int, int, int, const ColArgs&, int, hipStream_t);
template hipError_t launch_slab<double>(int, const SlabArgs&, int, hipStream_t);
}  // namespace fsp
