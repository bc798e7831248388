// Launchers of the allocation-free mass balance (hlb_noalloc.hip).  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "hlb_internal.h"

namespace hlb {

// Partial sums the allocation-free reduction holds per device (the context's
// own reduction uses as many): 64 KiB of device memory per GPU, kept until
// the process ends.
constexpr int64_t kNoAllocPartials = 8192;

// Looks up, once per device, the device address of the fixed partial-sum
// array (with the calling thread's current device) and returns it in *addr
// (may be null).
hipError_t noalloc_setup(double **addr);
// out[0] := offset + sum of the stored values of buffer `src` (the total
// mass), out[1] := out[0] - m0 - d.acc[0] (the balance residual); out is
// device memory.  Allocates nothing; asynchronous on `s`.
hipError_t launch_mass_balance_noalloc(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src,
                                       double offset, double m0, double *out, hipStream_t s);

}  // namespace hlb
