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
// Bulk+wall group pull table: positions [0, n0) are cut into segments of
// consecutive positions whose 18 incoming links have the same source offsets
// (source position minus own position; a wall link's offset is np, which
// puts the source outside [0, np): the link then reads the site's own slot
// of direction opp(i)).
// Each segment stores its offsets once, as a row of kSegRow int32 (18 used,
// padded for 16-byte loads); each position stores a one-byte segment index
// relative to the first segment of its kSegBlock-position block.
constexpr int kSegRow = 20;
constexpr int64_t kSegBlock = 256;
// Population buffers are tiled: positions are cut into tiles of kPopTile
// consecutive positions and a tile stores its 19 direction runs one after
// the other, [np / kPopTile][19][kPopTile].  Every wavefront still reads and
// writes 64 consecutive elements per direction, but the 38 streams of a step
// land in one region of memory instead of 38 regions np elements apart,
// which HBM serves at a higher rate.  np is a multiple of kPopTile.
constexpr int kPopTileShift = 12;
constexpr int64_t kPopTile = int64_t(1) << kPopTileShift;

struct IoletDev {
  int32_t kind;     // HLB_IOLET_VELOCITY / HLB_IOLET_PRESSURE
  int32_t tab_len;  // >= 1
  int64_t tab_off;  // offset into the concatenated table array
  double n[3];      // unit normal into the fluid
  int32_t wk;       // 1: a Windkessel outlet (density from wk_rho, outflow accumulated)
  int32_t pad;
};

// Windkessel outlet state: rho_k(s+1) = rho_ref + R1 Q_k(s) + X(s+1),
// X(s+1) = X(s) + (Q_k(s) - X(s)/R2)/C (C > 0; no leak if R2 = 0), or
// R2 Q_k(s) (C = 0); Q_k(s) the outflow of the update s -> s+1.
struct WkParams {
  double rho_ref, R1, C, R2, X, Q;
};

struct Layout {
  int64_t n_sites = 0;
  int64_t np = 0;               // padded site count (multiple of kPopTile)
  int64_t gbeg[kGroups + 1] = {0};
  int64_t gcnt[kGroups] = {0};
  int64_t io_begin = 0;         // first position of the iolet groups
  int64_t nio = 0;              // np - io_begin
  int64_t nseg = 0;             // segments of the bulk+wall group
  int64_t edge_blocks = 0;      // leading 256-position blocks of the bulk+wall group
                                // holding its edge sites (split step)
  int64_t ghost_begin = 0;      // positions [ghost_begin, ghost_begin + n_ghost):
  int64_t n_ghost = 0;          // copies of a peer partition's sites (no update)
};

struct DevPtrs {
  void *f[2] = {nullptr, nullptr};  // population buffers, [np/kPopTile][19][kPopTile] of the storage type
  int32_t *seg_off = nullptr;       // [nseg + 1][kSegRow] bulk+wall source offsets per segment
                                    // (the last row is padding, read by scalar row loads)
  int32_t *seg_base = nullptr;      // [ceil(n0 / kSegBlock)] first segment of each block
  uint8_t *seg_delta = nullptr;     // [n0] segment of each position minus its block's first
  int32_t *nbr_io = nullptr;        // iolet groups' pull table [18][nio]: source position of
                                    // population i (i = 1..18), or the link code (< 0)
  int32_t *order = nullptr;         // [np] caller id of each position (-1 for padding)
  double *corr = nullptr;           // [18][nio] Ladd coefficients of iolet-group links
  IoletDev *io = nullptr;           // [n_iolets]
  double *tables = nullptr;         // concatenated per-step iolet tables
  double *phi = nullptr;            // [np] porosity, or null
  double *acc = nullptr;            // [4] FP64 accumulators: boundary flux since t0, ...
  double *partial = nullptr;        // [partial_len] reduction scratch
  int64_t partial_len = 0;
  double *io_scratch = nullptr;     // [np*19] host-exchange staging (allocated lazily)
  double *wk_rho = nullptr;         // [n_iolets][2] Windkessel densities by time parity
  double *io_flux = nullptr;        // [n_iolets] outflow of the current update (Windkessel outlets)
  WkParams *wk = nullptr;           // [n_iolets]
  // Set only in the copies a replayed graph is captured with: the kernels
  // then take the time as *t_base + t (t = the step's index in the graph),
  // so that one graph serves every starting time.
  const int64_t *t_base = nullptr;
};

struct LaunchCfg {
  int storage = HLB_F64;
  double tau = 0.8;
  double rho0 = 1.0;
  int xcd_chunk = 0;  // blocks per XCD chunk (0: plain block order)
  bool porous = false;
  int scheme = HLB_SCHEME_PULL;
  int sites_per_thread = 1;  // bulk+wall sites per thread in the full pull step (1 or 2)
  bool ladd_local = false;   // Ladd rule with the site's own density (hlb_options.ladd_rho_local)
};

// Bulk+wall sites per thread of the full pull step for a storage type when
// the caller leaves it open (the measured best).
int default_sites_per_thread(int storage);

// ---- launchers (hlb_kernels.hip); all asynchronous on `s` ----
// One update t -> t+1: reads buffer `src`, writes buffer 1-src.
// ev_begin / ev_end (may be null) are recorded around the step kernel.
hipError_t launch_step(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, int64_t t,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1, int part = 0);
// Halo pack (pack = true: buffer `buf` -> io) or unpack (io -> buffer `buf`)
// of n (position, direction) values.
hipError_t launch_halo(const LaunchCfg &cfg, const DevPtrs &d, int buf, const int32_t *pos, const int32_t *dir,
                       int64_t n, void *io, bool pack, hipStream_t s);
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
// After the update t -> t+1: Windkessel outlets take their outflow, advance
// their state and set the density of the update t+1 -> t+2; the outflow
// accumulators are cleared (no memset: the launch may be graph-captured).
hipError_t launch_windkessel(const DevPtrs &d, int n_io, int64_t t, hipStream_t s);
// *p = v, and *p += k (one thread each; a kernel, not a memset, so that the
// second can sit in a captured graph).
hipError_t launch_set_time(int64_t *p, int64_t v, hipStream_t s);
hipError_t launch_add_time(int64_t *p, int64_t k, hipStream_t s);
// Sum of the stored deviations of buffer `src` into d.partial[0] (FP64).
hipError_t launch_mass(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src,
                       hipStream_t s);

}  // namespace hlb
