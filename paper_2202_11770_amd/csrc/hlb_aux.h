// Launchers of the auxiliary kernels (hlb_aux.hip).  Not part of the public
// ABI; all asynchronous on `s`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hlb {

// Rules of launch_check_values.
enum { kCheckFinite = 0, kCheckPositive = 1, kCheckUnit = 2 };

// *flag := 1 if any of v[0..n) breaks the rule (finite; finite and > 0;
// in [0, 1]), else 0.  v and flag are device pointers.
hipError_t launch_check_values(const double *v, int64_t n, int mode, int32_t *flag, hipStream_t s);
// pos[p] := caller[order[p]] (0 where order[p] < 0), p in [0, np).
hipError_t launch_from_caller(const double *caller, const int32_t *order, int64_t np, double *pos, hipStream_t s);
// caller[order[p]] := pos[p] where order[p] >= 0, p in [0, np).
hipError_t launch_to_caller(const double *pos, const int32_t *order, int64_t np, double *caller, hipStream_t s);

}  // namespace hlb
