// Internal declarations shared by the host runtime (hlb_runtime.cpp) and the
// gfx950 kernels (hlb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hlb.h"

namespace hlb {

// Number of site groups that get their own range (Sec. 3.2.2): the merged
// bulk+wall group, then inlet, outlet, inlet+wall, outlet+wall.
constexpr int kGroups = 5;
// Each group range starts on a multiple of this many sites, so that no
// 64-lane wavefront straddles two groups (wavefront-uniform code paths).
constexpr int64_t kGroupAlign = 256;

struct IoletDev {
  int32_t kind;     // HLB_IOLET_VELOCITY / HLB_IOLET_PRESSURE
  int32_t tab_len;  // >= 1
  int64_t tab_off;  // offset into the concatenated table array
  double n[3];      // unit normal into the fluid
  double pad;
};

struct Layout {
  int64_t n_sites = 0;
  int64_t np = 0;               // padded site count = stride of one direction array
  int64_t gbeg[kGroups + 1] = {0};
  int64_t gcnt[kGroups] = {0};
  int64_t io_begin = 0;         // first position of the iolet groups
  int64_t nio = 0;              // np - io_begin
};

struct DevPtrs {
  void *f[2] = {nullptr, nullptr};  // population buffers, [19][np] of the storage type
  int32_t *nbr = nullptr;           // pull table [18][np]: source position of population i
                                    // (i = 1..18), or the link code (< 0)
  int32_t *order = nullptr;         // [np] caller id of each position (-1 for padding)
  double *corr = nullptr;           // [18][nio] Ladd coefficients of iolet-group links
  IoletDev *io = nullptr;           // [n_iolets]
  double *tables = nullptr;         // concatenated per-step iolet tables
  double *phi = nullptr;            // [np] porosity, or null
  double *acc = nullptr;            // [4] FP64 accumulators: boundary flux since t0, ...
  double *partial = nullptr;        // [partial_len] reduction scratch
  int64_t partial_len = 0;
  double *io_scratch = nullptr;     // [np*19] host-exchange staging (allocated lazily)
};

struct LaunchCfg {
  int storage = HLB_F64;
  double tau = 0.8;
  double rho0 = 1.0;
  bool xcd_remap = true;
  bool porous = false;
};

// ---- launchers (hlb_kernels.hip); all asynchronous on `s` ----
// One update t -> t+1: reads buffer `src`, writes buffer 1-src.
hipError_t launch_step(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, int64_t t,
                       hipStream_t s, hipEvent_t ev_bulk_begin, hipEvent_t ev_bulk_end,
                       hipEvent_t ev_io_end);
// Both buffers := equilibrium of (rho, u) given per caller id in staging
// (staging: [n][4] doubles rho, ux, uy, uz) or rest if staging is null.
hipError_t launch_init_eq(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d,
                          const double *staging, hipStream_t s);
// Pre-collision populations of time t.  direct: buffer `src` already holds
// them; otherwise they are gathered from buffer `src` (post-collision, t-1)
// with the boundary rules of step t-1.  Writes, per caller id, rho/u/wss
// (any null) or, if f_out is non-null, the [n][19] unshifted populations.
hipError_t launch_macros(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, bool direct,
                         int64_t t_prev, double *rho, double *u, double *wss, double *f_out,
                         hipStream_t s);
// Set pre-collision state from staging [n][19] (caller order, unshifted):
// buffer `pre` := f - w rho0, buffer 1-pre := its collision.
hipError_t launch_set_state(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int pre,
                            const double *staging, hipStream_t s);
// p[0..n) := 0 (a kernel, so that no memset node lands in a captured graph).
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);
// Sum of the stored deviations of buffer `src` into d.partial[0] (FP64).
hipError_t launch_mass(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src,
                       hipStream_t s);

}  // namespace hlb
