// Row-pass launchers (double): every length and schedule variant of P1 and P5.
#include "solve_launch.hpp"

namespace fsp {
template hipError_t launch_p1<double>(int, int, const RowArgs&, int, hipStream_t);
template hipError_t launch_p5<double>(int, int, const RowArgs&, int, hipStream_t);
}  // namespace fsp
