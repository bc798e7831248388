// Launchers of the adjoint sweep beyond those in hlb_internal.h (hlb_adjoint.hip).
// Not part of the public ABI.
#pragma once

#include "hlb_internal.h"

namespace hlb {

// The objective buffer b.J holds the objective at [0], the caller's flux
// accumulators while a sweep runs at [1, 5), and from kAdjJPart on one
// partial objective sum per 256-position workgroup of the collide kernel
// (adj_jpart_slots(np) of them), which a sweep starts at zero.
constexpr int64_t kAdjJPart = 8;
inline int64_t adj_jpart_slots(int64_t np) { return (np + 255) / 256; }
// After the last adjoint step of a sweep: J[0] += the workgroups' partial sums.
hipError_t launch_adjoint_finish(const AdjBuffers &b, int64_t np, hipStream_t s);

}  // namespace hlb
