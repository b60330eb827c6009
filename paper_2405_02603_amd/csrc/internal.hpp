// internal.hpp -- library-internal calls between the plan code (api.hip) and
// the serving engine (serve_engine.hip); not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "fsp.h"

namespace fsp {
namespace internal {

// count solves that share the geometry, schedule and twiddle tables of plan
// `geo` (same grid and precision): solve i reads rho[i], writes phi[i], uses the
// workspace work[i] (work1_bytes) and the Green's octant octant[i] (of any plan
// of this grid and precision).  Up to 16 solves share each launch.
hipError_t solve_items(fsp_plan geo, int count, const void* const* rho, void* const* phi, void* const* work,
                       const void* const* octant, hipStream_t s);

size_t work1_bytes(fsp_plan p);       // one spectrum's workspace
size_t ghat_bytes(fsp_plan p);        // the Green's buffer
size_t precompute_bytes(fsp_plan p);  // transient bytes of fsp_precompute
const void* octant(fsp_plan p);       // the Green's octant of a precomputed plan

// Bind only a (caller-owned) Green's buffer: the plan can be precomputed and its
// octant read, but not solved.
fsp_status bind_ghat(fsp_plan p, void* ghat_dev);

const char* last_error();
void set_error(const std::string& msg);  // the text fsp_last_error() returns on this thread

}  // namespace internal
}  // namespace fsp
