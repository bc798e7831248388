// gfx950 kernels of the sparse D3Q19 LBGK update (pull scheme).
//
// One thread owns one fluid site.  Populations live in two buffers (f_old /
// f_new swapped by pointer, Sec. 3.2.3), each a structure of arrays per
// tile of 4096 positions, [np/4096][19][4096] of the storage type.  FP64
// stores f_i itself, as the paper does; the FP32 / FP16 forms store the
// deviation f_i - w_i rho0 from the rest state and collide in FP32.  A step gathers the 19
// post-collision populations that stream into the site (eq. (3b) read
// backwards: the pull order the paper proposes in its future-work section),
// substitutes the boundary rules for links that cross a wall or an iolet
// (Sec. 2.3), collides (eq. (3a) with eq. (4)) and stores the 19 results at
// the site's own, coalesced, slots.
//
// Sites are grouped by collision-streaming type (Sec. 3.2.2): positions
// [0, n0) hold the merged bulk+wall group, whose pull table encodes
// bounce-back as one load with a selected address; the four iolet groups follow, each
// starting on a 256-site boundary, with the boundary rules applied per link.
// k_step runs both code paths in one launch, one group per workgroup.
//
// The method is bound by HBM bandwidth (~0.7 flop per byte in FP64), so
// nothing here uses the matrix cores.

#include "hlb_device.h"

namespace hlb {
namespace {

using namespace dev;

// ---------------------------------------------------------------- step ----

// One launch per step covers every group (Sec. 3.2.2's per-type kernels as
// block-uniform code paths of a single launch): the first nb_io blocks take
// the iolet groups, so that their longer-latency work starts first and
// overlaps the bulk blocks; the remaining nb_bulk blocks take the bulk+wall
// group's 256-position blocks blk0, blk0+1, ...  (a split step launches the
// edge blocks and the rest separately).  Every block, hence every wavefront,
// runs one group's code path only.
// Per storage type, measured on the 2e7-site tree: the minimum waves per
// SIMD the step kernel is compiled for (the rare iolet blocks spill to fit,
// the bulk path does not), and whether population addresses use 32-bit byte
// offsets when a buffer allows it (see at()).  FP64: the natural 4 waves and
// 32-bit offsets; FP32: 6 waves and 64-bit addresses (32-bit offsets
// measured 3% slower); FP16: 6 waves and 32-bit offsets.  Measured again
// with the per-storage workgroup-to-XCD chunk on the 2e7- and 2e8-site
// trees: FP64 4 waves (5, 6 slower by 0.5-1% on the 2e8 tree), FP16 6 (8
// waves 0.5-1.6% slower, 5 waves 2-3%).  FP32, with the segment rows in LDS
// and the banded order: 6 waves against its natural 5 gave +0.2-0.3% on the
// trees and +0.9-1.0% on the 6e8-site forest; 4 waves cost 5%.
// SPT = 2 (two bulk+wall sites per thread, see below) needs about twice the
// registers of the bulk path: 4 waves.
template <typename T, int SPT = 1, bool NARROW = true>
constexpr int kStepWaves = SPT == 2 ? 4 : (std::is_same<T, double>::value ? 4 : 6);
template <typename T>
constexpr bool kStepNarrow = !std::is_same<T, float>::value;
// Whether the bulk path stages each block's segment rows through LDS: one
// coalesced pass over the block's rows (typically 20-50 of them) replaces
// every lane's five 16-byte row loads, each of which touches a cache line
// per distinct segment of its wavefront.  FP64 and FP32: +0.4% on the 2e7-
// and +0.5-1.3% on the 2e8-site tree.  FP16 keeps its wavefront-wide scalar
// row loads: the staging pass and barrier cost it 3-5%.
template <typename T>
constexpr bool kStepLdsRows = sizeof(T) != 2;

// SPT: bulk+wall sites per thread.  With SPT = 2 a workgroup takes two
// consecutive 256-position blocks and each thread one position of each (both
// coalesced); the two sites' table loads and 36 gathers are all issued
// before either collides, which doubles the bytes a wavefront has in flight.
// nb_bulk then counts block pairs.  Only the full step (blk0 = 0) uses it.
template <typename T, bool POROUS, bool NARROW, int SPT = 1>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kStepWaves<T, SPT, NARROW>, 8))) void k_step(
    const T *__restrict__ A, T *__restrict__ B, GatherArgs a, const int32_t *__restrict__ order, int64_t n0,
    int64_t nb_io, int64_t blk0, int64_t nb_bulk, int xcd_chunk, typename Acc<T>::type omega, double *acc) {
  using C = typename Acc<T>::type;
  constexpr bool SH = kShifted<T>;
  const int64_t b = blockIdx.x;
  C flux = 0;
  if (b < nb_io) {
    const int64_t p = a.io_begin + b * kBlock + threadIdx.x;
    WkFlux wkf;
    if (p < a.np && order[p] >= 0) {
      C g[Q];
      flux = gather<true, POROUS, SH, NARROW>(A, p, 0, a, g, &wkf);
      collide<SH>(g, omega, C(a.rho0));
#pragma unroll
      for (int i = 0; i < Q; ++i) st(at<NARROW>(B, (int32_t)p, i), g[i]);
    }
    const double s = wave_sum(double(flux));
    if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(acc, s);
    if (a.io_flux) wave_add_grouped(a.io_flux, wkf);
  } else if constexpr (SPT == 1) {
    const int64_t blk = blk0 + block_id(b - nb_io, nb_bulk, xcd_chunk);
    const int64_t p = blk * kBlock + threadIdx.x;
    constexpr bool LROWS = kStepLdsRows<T>;
    // rows of the block's segments: seg_base[blk] .. + seg_delta of its last
    // position (at most kSegBlock rows)
    __shared__ int4 lrows[LROWS ? kSegBlock * (kSegRow / 4) : 1];
    int32_t k_row = 0;
    if constexpr (LROWS) {
      // p's row in the block, loaded before the pass so that the two loads'
      // latencies overlap (no load moves across the barrier)
      k_row = p < n0 ? (int32_t)ld_stream(a.seg_delta + p) : 0;
      const int64_t last = blk * kBlock + kBlock - 1 < n0 ? blk * kBlock + kBlock - 1 : n0 - 1;
      const int32_t n4 = ((int32_t)a.seg_delta[last] + 1) * (kSegRow / 4);
      const int4 *rows = reinterpret_cast<const int4 *>(a.seg_off + (int64_t)a.seg_base[blk] * kSegRow);
      for (int k = threadIdx.x; k < n4; k += kBlock) lrows[k] = rows[k];
      __syncthreads();
    }
    if (p < n0) {
      C g[Q];
      flux = gather<false, POROUS, SH, NARROW, LROWS>(A, p, blk, a, g, nullptr, lrows + (kSegRow / 4) * k_row);
      collide<SH>(g, omega, C(a.rho0));
      if constexpr (NARROW) {
        using N = Narrow<T>;
        const uint32_t own = N::voff(((uint32_t)p << N::S) + N::D);
#pragma unroll
        for (int i = 0; i < Q; ++i) st(N::at(B, i, own), g[i]);
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) st(at<NARROW>(B, (int32_t)p, i), g[i]);
      }
    }
    if constexpr (POROUS) {
      const double s = wave_sum(double(flux));
      if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(acc, s);
    }
  } else {
    const int64_t blk = 2 * block_id(b - nb_io, nb_bulk, xcd_chunk);
    const int64_t p = blk * kBlock + threadIdx.x;
    if (p < n0) {
      // the second site; past the group's end (last pair only) it repeats
      // the first and stores the same values again (a conditional store
      // would let the compiler sink the second site's loads behind the
      // first site's stores)
      const bool has2 = p + kBlock < n0;
      const int64_t p2 = has2 ? p + kBlock : p, blk2 = has2 ? blk + 1 : blk;
      C g[Q], h[Q], flux2;
      gather_bulk2<POROUS, SH, NARROW>(A, p, blk, p2, blk2, a, g, h, flux, flux2);
      if (has2) flux += flux2;
      collide<SH>(g, omega, C(a.rho0));
      collide<SH>(h, omega, C(a.rho0));
#pragma unroll
      for (int i = 0; i < Q; ++i) st(at<NARROW>(B, (int32_t)p, i), g[i]);
#pragma unroll
      for (int i = 0; i < Q; ++i) st(at<NARROW>(B, (int32_t)p2, i), h[i]);
    }
    if constexpr (POROUS) {
      const double s = wave_sum(double(flux));
      if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(acc, s);
    }
  }
}

// One step in push order (the paper's implementation; the A/B partner of
// k_step): buffers hold the pre-collision state f(t); every site reads its
// own 19 values (coalesced), collides and scatters (scatter()).  Same block
// layout, XCD remap and occupancy as k_step.
template <typename T, bool POROUS, bool NARROW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kStepWaves<T>, 8))) void k_step_push(
    const T *__restrict__ A, T *__restrict__ B, GatherArgs a, const int32_t *__restrict__ order, int64_t n0,
    int64_t nb_io, int64_t blk0, int64_t nb_bulk, int xcd_chunk, typename Acc<T>::type omega, double *acc) {
  using C = typename Acc<T>::type;
  constexpr bool SH = kShifted<T>;
  const int64_t b = blockIdx.x;
  C flux = 0;
  if (b < nb_io) {
    const int64_t p = a.io_begin + b * kBlock + threadIdx.x;
    WkFlux wkf;
    if (p < a.np && order[p] >= 0) {
      C f[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = ld(at<NARROW>(A, (int32_t)p, i));
      C dr, rho, jx, jy, jz;
      moments<SH>(f, C(a.rho0), dr, rho, jx, jy, jz);
      collide<SH>(f, omega, C(a.rho0));
      flux = scatter<true, POROUS, SH, NARROW>(B, p, 0, a, f, jx / rho, jy / rho, jz / rho, rho, &wkf);
    }
    const double s = wave_sum(double(flux));
    if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(acc, s);
    if (a.io_flux) wave_add_grouped(a.io_flux, wkf);
  } else {
    const int64_t blk = blk0 + block_id(b - nb_io, nb_bulk, xcd_chunk);
    const int64_t p = blk * kBlock + threadIdx.x;
    if (p < n0) {
      C f[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = ld(at<NARROW>(A, (int32_t)p, i));
      collide<SH>(f, omega, C(a.rho0));
      flux = scatter<false, POROUS, SH, NARROW>(B, p, blk, a, f, C(0), C(0), C(0), C(0));
    }
    if constexpr (POROUS) {
      const double s = wave_sum(double(flux));
      if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(acc, s);
    }
  }
}

// ------------------------------------------------------- init / state ----

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_eq(T *__restrict__ A, T *__restrict__ B,
                                                    const int32_t *__restrict__ order, int64_t np,
                                                    const double *__restrict__ staging, double rho0) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  const int32_t id = order[p];
  constexpr bool SH = kShifted<T>;
  double g[Q];
  if (id < 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = 0.0;
  } else if (staging == nullptr) {
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = rest<SH>(i, rho0);
  } else {
    const double rho = staging[4 * (int64_t)id], ux = staging[4 * (int64_t)id + 1],
                 uy = staging[4 * (int64_t)id + 2], uz = staging[4 * (int64_t)id + 3];
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = s_eq<SH>(i, rho - rho0, rho, ux, uy, uz, usq);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    st(A + pidx((int32_t)p, i), static_cast<typename Acc<T>::type>(g[i]));
    st(B + pidx((int32_t)p, i), static_cast<typename Acc<T>::type>(g[i]));
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_state(T *__restrict__ Pre, T *__restrict__ Post,
                                                      const int32_t *__restrict__ order, int64_t np,
                                                      const double *__restrict__ staging, double rho0,
                                                      typename Acc<T>::type omega) {
  using C = typename Acc<T>::type;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  const int32_t id = order[p];
  constexpr bool SH = kShifted<T>;
  C g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i)
    g[i] = id < 0 ? C(0) : C(staging[(int64_t)id * Q + i] - shift<SH>(i, rho0));
#pragma unroll
  for (int i = 0; i < Q; ++i) st(Pre + pidx((int32_t)p, i), g[i]);
  if (id < 0) return;
  collide<SH>(g, omega, C(rho0));
#pragma unroll
  for (int i = 0; i < Q; ++i) st(Post + pidx((int32_t)p, i), g[i]);
}

// --------------------------------------------------------------- macros ----

// Density, velocity, wall shear stress (or the populations) of the
// pre-collision state at time t, in FP64, written per caller id.
template <typename T, bool POROUS>
__global__ __launch_bounds__(kBlock) void k_macros(const T *__restrict__ A, GatherArgs a,
                                                   const int32_t *__restrict__ order, int direct,
                                                   double tau, double *rho_o, double *u_o,
                                                   double *wss_o, double *f_o) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= a.np) return;
  const int32_t id = order[p];
  if (id < 0) return;
  constexpr bool SH = kShifted<T>;
  double g[Q];
  if (direct) {
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = ld(A + pidx((int32_t)p, i));
  } else if (p < a.io_begin) {
    gather<false, POROUS, SH>(A, p, p / kBlock, a, g);
  } else {
    gather<true, POROUS, SH>(A, p, 0, a, g);
  }
  if (f_o) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f_o[(int64_t)id * Q + i] = g[i] + shift<SH>(i, a.rho0);
    return;
  }
  double dr, rho, jx, jy, jz;
  moments<SH>(g, a.rho0, dr, rho, jx, jy, jz);
  const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  if (rho_o) rho_o[id] = rho;
  if (u_o) {
    u_o[3 * (int64_t)id] = ux;
    u_o[3 * (int64_t)id + 1] = uy;
    u_o[3 * (int64_t)id + 2] = uz;
  }
  if (!wss_o) return;
  // wall normal: normalised sum of the directions whose links hit a wall;
  // pull entry i describes the link leaving along opp(i) = -c_i (a wall
  // link is coded -1 in the iolet groups, outside [0, np) in the bulk group)
  double nx = 0, ny = 0, nz = 0;
  bool any = false;
  const bool bulk = p < a.io_begin;
  int32_t off[Q - 1];
  if (bulk) bulk_offsets(a, p, p / kBlock, off);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const bool wall = bulk ? (uint64_t)(p + (int64_t)off[i - 1]) >= (uint64_t)a.np
                           : a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)] == HLB_LINK_WALL;
    if (wall) {
      any = true;
      nx -= cx(i);
      ny -= cy(i);
      nz -= cz(i);
    }
  }
  double w = 0.0;
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  if (any && nn > 0.0) {
    nx /= nn;
    ny /= nn;
    nz /= nn;
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
    double pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // non-equilibrium part f - f_eq (the same in either representation)
      const double d = g[i] - s_eq<SH>(i, dr, rho, ux, uy, uz, usq);
      pxx += d * cx(i) * cx(i);
      pyy += d * cy(i) * cy(i);
      pzz += d * cz(i) * cz(i);
      pxy += d * cx(i) * cy(i);
      pxz += d * cx(i) * cz(i);
      pyz += d * cy(i) * cz(i);
    }
    const double fac = -(1.0 - 1.0 / (2.0 * tau));
    const double tx = fac * (pxx * nx + pxy * ny + pxz * nz);
    const double ty = fac * (pxy * nx + pyy * ny + pyz * nz);
    const double tz = fac * (pxz * nx + pyz * ny + pzz * nz);
    const double tn = tx * nx + ty * ny + tz * nz;
    const double sx = tx - tn * nx, sy = ty - tn * ny, sz = tz - tn * nz;
    w = sqrt(sx * sx + sy * sy + sz * sz);
  }
  wss_o[id] = w;
}

// ----------------------------------------------------------------- mass ----

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mass_partial(const T *__restrict__ A,
                                                         const int32_t *__restrict__ order, int64_t np,
                                                         double *partial) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < np; p += (int64_t)gridDim.x * kBlock) {
    if (order[p] < 0) continue;
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) q += ld(A + pidx((int32_t)p, i));
    s += q;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) b += red[w];
    partial[1 + blockIdx.x] = b;
  }
}

__global__ __launch_bounds__(kBlock) void k_mass_final(double *partial, int64_t nparts) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nparts; k += kBlock) s += partial[1 + k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) b += red[w];
    partial[0] = b;
  }
}

// One thread per iolet (see launch_windkessel).  t_base: as in GatherArgs.
__global__ void k_windkessel(const IoletDev *io, WkParams *wk, double *wk_rho, double *io_flux, int n_io,
                             int64_t t, const int64_t *t_base) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_io || !io[k].wk) return;
  if (t_base) t += *t_base;
  const double Q = io_flux[k];
  io_flux[k] = 0.0;
  WkParams P = wk[k];
  if (P.C > 0.0)
    P.X += (Q - (P.R2 > 0.0 ? P.X / P.R2 : 0.0)) / P.C;
  else
    P.X = P.R2 * Q;
  P.Q = Q;
  wk[k] = P;
  wk_rho[2 * k + ((t + 1) & 1)] = P.rho_ref + P.R1 * Q + P.X;
}

__global__ void k_set_time(int64_t *p, int64_t v) { *p = v; }
__global__ void k_add_time(int64_t *p, int64_t k) { *p += k; }

__global__ void k_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename T>
hipError_t step_impl(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, int64_t t,
                     hipStream_t s, hipEvent_t e0, hipEvent_t e1, int part) {
  using C = typename Acc<T>::type;
  const T *A = static_cast<const T *>(d.f[src]);
  T *B = static_cast<T *>(d.f[1 - src]);
  const GatherArgs a = make_args(cfg, L, d, t);
  const C omega = C(1.0 / cfg.tau);
  const int64_t n0 = L.gcnt[0];
  const int64_t nb_all = (n0 + kBlock - 1) / kBlock;
  // part 0: the whole step; 1: iolet groups + the edge blocks of the
  // bulk+wall group; 2: its remaining blocks
  const int64_t nb_io = part == 2 ? 0 : (L.nio + kBlock - 1) / kBlock;
  const int64_t blk0 = part == 2 ? L.edge_blocks : 0;
  const int64_t nb_bulk = part == 0 ? nb_all : (part == 1 ? L.edge_blocks : nb_all - L.edge_blocks);
  // two bulk+wall sites per thread: full pull steps only
  const bool pair = cfg.sites_per_thread == 2 && part == 0 && cfg.scheme == HLB_SCHEME_PULL;
  const int64_t nb_launch = pair ? (nb_bulk + 1) / 2 : nb_bulk;
  const unsigned grid = (unsigned)(nb_io + nb_launch);
  hipError_t er;
  if (e0 && (er = hipEventRecord(e0, s)) != hipSuccess) return er;
  // byte offsets fit in 32 bits when a whole population buffer does, with
  // the bias of the bulk path's addressing (Narrow)
  const bool narrow = kStepNarrow<T> && (uint64_t)Q * (uint64_t)L.np * sizeof(T) + Narrow<T>::BIAS <=
                                            (uint64_t(1) << 32);
  if (grid > 0) {
#define HLB_STEP(P, N)                                                                                    \
  do {                                                                                                  \
    if (cfg.scheme == HLB_SCHEME_PUSH)                                                                  \
      k_step_push<T, P, N><<<grid, kBlock, 0, s>>>(A, B, a, d.order, n0, nb_io, blk0, nb_bulk,          \
                                                   cfg.xcd_chunk, omega, d.acc);                        \
    else if (pair)                                                                                      \
      k_step<T, P, N, 2><<<grid, kBlock, 0, s>>>(A, B, a, d.order, n0, nb_io, 0, nb_launch,             \
                                                 cfg.xcd_chunk, omega, d.acc);                          \
    else                                                                                                \
      k_step<T, P, N><<<grid, kBlock, 0, s>>>(A, B, a, d.order, n0, nb_io, blk0, nb_bulk, cfg.xcd_chunk, \
                                              omega, d.acc);                                            \
  } while (0)
    if (cfg.porous) {
      if (narrow) HLB_STEP(true, kStepNarrow<T>);
      else HLB_STEP(true, false);
    } else {
      if (narrow) HLB_STEP(false, kStepNarrow<T>);
      else HLB_STEP(false, false);
    }
#undef HLB_STEP
  }
  if ((er = hipGetLastError()) != hipSuccess) return er;
  if (e1 && (er = hipEventRecord(e1, s)) != hipSuccess) return er;
  return hipSuccess;
}

// Halo exchange (one-GPU emulation of the domain split; the same kernels
// serve a multi-GPU run): pack copies the listed (position, direction)
// values of a population buffer into a contiguous buffer, unpack writes a
// contiguous buffer into the listed slots.  Raw stored values, no rounding.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack(const T *__restrict__ A, const int32_t *__restrict__ pos,
                                                 const int32_t *__restrict__ dir, int64_t n, T *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) out[k] = A[pidx(pos[k], dir[k])];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_unpack(T *__restrict__ A, const int32_t *__restrict__ pos,
                                                   const int32_t *__restrict__ dir, int64_t n,
                                                   const T *__restrict__ in) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) A[pidx(pos[k], dir[k])] = in[k];
}

template <typename T>
hipError_t halo_impl(const DevPtrs &d, int buf, const int32_t *pos, const int32_t *dir, int64_t n, void *io,
                     bool pack, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (pack)
    k_pack<T><<<blocks_for(n), kBlock, 0, s>>>(static_cast<const T *>(d.f[buf]), pos, dir, n, static_cast<T *>(io));
  else
    k_unpack<T><<<blocks_for(n), kBlock, 0, s>>>(static_cast<T *>(d.f[buf]), pos, dir, n,
                                                 static_cast<const T *>(io));
  return hipGetLastError();
}

template <typename T>
hipError_t macros_impl(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, bool direct,
                       int64_t t_prev, double *rho, double *u, double *wss, double *f_out,
                       hipStream_t s) {
  const T *A = static_cast<const T *>(d.f[src]);
  GatherArgs a = make_args(cfg, L, d, t_prev < 0 ? 0 : t_prev);
  a.io_flux = nullptr;  // the re-gather does not count towards the outflow
  if (cfg.porous)
    k_macros<T, true><<<blocks_for(L.np), kBlock, 0, s>>>(A, a, d.order, direct ? 1 : 0, cfg.tau, rho, u,
                                                          wss, f_out);
  else
    k_macros<T, false><<<blocks_for(L.np), kBlock, 0, s>>>(A, a, d.order, direct ? 1 : 0, cfg.tau, rho, u,
                                                           wss, f_out);
  return hipGetLastError();
}

template <typename T>
hipError_t init_impl(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, const double *staging,
                     hipStream_t s) {
  k_init_eq<T><<<blocks_for(L.np), kBlock, 0, s>>>(static_cast<T *>(d.f[0]), static_cast<T *>(d.f[1]),
                                                   d.order, L.np, staging, cfg.rho0);
  return hipGetLastError();
}

template <typename T>
hipError_t set_state_impl(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int pre,
                          const double *staging, hipStream_t s) {
  using C = typename Acc<T>::type;
  k_set_state<T><<<blocks_for(L.np), kBlock, 0, s>>>(static_cast<T *>(d.f[pre]), static_cast<T *>(d.f[1 - pre]),
                                                     d.order, L.np, staging, cfg.rho0, C(1.0 / cfg.tau));
  return hipGetLastError();
}

template <typename T>
hipError_t mass_impl(const Layout &L, const DevPtrs &d, int src, hipStream_t s) {
  int64_t nb = blocks_for(L.np);
  if (nb > d.partial_len - 1) nb = d.partial_len - 1;
  k_mass_partial<T><<<(unsigned)nb, kBlock, 0, s>>>(static_cast<const T *>(d.f[src]), d.order, L.np, d.partial);
  k_mass_final<<<1, kBlock, 0, s>>>(d.partial, nb);
  return hipGetLastError();
}

}  // namespace

#define HLB_DISPATCH(storage, CALL)                       \
  switch (storage) {                                      \
    case HLB_F64: { using T = double; return CALL; }      \
    case HLB_F32_SHIFTED: { using T = float; return CALL; } \
    case HLB_F16_SHIFTED: { using T = _Float16; return CALL; } \
    default: return hipErrorInvalidValue;                 \
  }

int default_sites_per_thread(int storage) {
  (void)storage;
  return 1;
}

hipError_t launch_step(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, int64_t t,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1, int part) {
  HLB_DISPATCH(cfg.storage, step_impl<T>(cfg, L, d, src, t, s, e0, e1, part));
}

hipError_t launch_halo(const LaunchCfg &cfg, const DevPtrs &d, int buf, const int32_t *pos, const int32_t *dir,
                       int64_t n, void *io, bool pack, hipStream_t s) {
  HLB_DISPATCH(cfg.storage, halo_impl<T>(d, buf, pos, dir, n, io, pack, s));
}

hipError_t launch_init_eq(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, const double *staging,
                          hipStream_t s) {
  HLB_DISPATCH(cfg.storage, init_impl<T>(cfg, L, d, staging, s));
}

hipError_t launch_macros(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, bool direct,
                         int64_t t_prev, double *rho, double *u, double *wss, double *f_out, hipStream_t s) {
  HLB_DISPATCH(cfg.storage, macros_impl<T>(cfg, L, d, src, direct, t_prev, rho, u, wss, f_out, s));
}

hipError_t launch_set_state(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int pre,
                            const double *staging, hipStream_t s) {
  HLB_DISPATCH(cfg.storage, set_state_impl<T>(cfg, L, d, pre, staging, s));
}

hipError_t launch_windkessel(const DevPtrs &d, int n_io, int64_t t, hipStream_t s) {
  if (n_io <= 0 || !d.wk) return hipSuccess;
  k_windkessel<<<(n_io + 63) / 64, 64, 0, s>>>(d.io, d.wk, d.wk_rho, d.io_flux, n_io, t, d.t_base);
  return hipGetLastError();
}

hipError_t launch_set_time(int64_t *p, int64_t v, hipStream_t s) {
  k_set_time<<<1, 1, 0, s>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_add_time(int64_t *p, int64_t k, hipStream_t s) {
  k_add_time<<<1, 1, 0, s>>>(p, k);
  return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_zero<<<blocks_for(n), kBlock, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_mass(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, hipStream_t s) {
  HLB_DISPATCH(cfg.storage, mass_impl<T>(L, d, src, s));
}

}  // namespace hlb
