// Row-pass launchers (float): every length and schedule variant of P1 and P5.
#include "solve_launch.hpp"

namespace fsp {
template hipError_t launch_p1<float>(int, int, const RowArgs&, int, hipStream_t);
template hipError_t launch_p5<float>(int, int, const RowArgs&, int, hipStream_t);
}  // namespace fsp
