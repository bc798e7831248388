// Launchers and device buffers of the adjoint sweep (hlb_adjoint.hip).  Not
// part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hlb_internal.h"

namespace hlb {

// Partial sums of the objective: each wavefront adds its share to slot
// (wavefront index mod kAdjJSlots), so that no single address takes one
// atomic per wavefront of the grid.
constexpr int64_t kAdjJSlots = 4096;
// Length of AdjBuffers::J: [0] the objective, [1, 5) the caller's flux
// accumulators while a sweep runs, [8, 8 + kAdjJSlots) the partial sums.
constexpr int64_t kAdjJLen = 8 + kAdjJSlots;

// Device buffers of the adjoint sweep (FP64 storage only).
struct AdjBuffers {
  double *mu = nullptr;       // adjoint of the post-collision state (tiled, as the state)
  double *nu = nullptr;       // adjoint of the pre-collision state (tiled, as the state)
  double *J = nullptr;        // [kAdjJLen] objective, saved flux accumulators, partial sums
  double *dA = nullptr;       // [n_iolets][n_steps]
  double *dphi = nullptr;     // [np] porosity derivative per position
  int32_t *blist = nullptr;   // positions of the sites with wall or iolet links, ascending
  int64_t n_blist = 0;
  int64_t n_blist_wall = 0;   // leading entries below the iolet groups (wall links only)
  int32_t objective = HLB_OBJ_WSS;
  double *w = nullptr;        // [n_iolets] iolet-flux weights (device)
  int32_t n_io = 0;           // iolets
  double *wq = nullptr;       // [n_iolets] outflow weights of the reverse step in flight
  double *lamX = nullptr;     // [n_iolets] adjoint of the Windkessel outlets' X
};
// Adjoint of the update (t-1 -> t): buffer `src` holds s_{t-1}; b.mu holds
// mu_t on entry and mu_{t-1} on return; accumulates J's partial sums (if
// in_window), the iolet table-value derivatives into column `step` of dA
// and the porosity derivatives.
hipError_t launch_adjoint_step(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, int64_t t,
                               const AdjBuffers &b, int in_window, int64_t n_steps, int64_t step,
                               hipStream_t s);
// The outflow weights b.wq of the reverse step of the update
// t0 + step -> t0 + step + 1 (run first in each reverse step by
// launch_adjoint_step; b.lamX must be zero before the sweep's first step).
// J[0] := sum of the partial sums J[8, 8 + kAdjJSlots) (one workgroup).
hipError_t launch_adjoint_objective(double *J, hipStream_t s);

}  // namespace hlb
