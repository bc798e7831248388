// Device-side building blocks of the sparse D3Q19 LBGK update, shared by the
// forward step kernels (hlb_kernels.hip) and the adjoint kernels
// (hlb_adjoint.hip): lattice constants, storage conversions, moments,
// equilibrium, BGK collision and the pull gather with the boundary rules.
#pragma once

#include <type_traits>

#include "hlb_internal.h"

namespace hlb {
namespace dev {

constexpr int Q = 19;
constexpr int kBlock = 256;

// D3Q19, opposite directions adjacent (the input convention of hlb.h).
__host__ __device__ constexpr int cx(int i) {
  constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return v[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return v[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return v[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// weights 1/3, 1/18, 1/36 (Sec. 2.2)
template <typename C>
__host__ __device__ constexpr C wgt(int i) {
  return i == 0 ? C(1) / C(3) : (i <= 6 ? C(1) / C(18) : C(1) / C(36));
}

// Compute type: double for FP64 storage, float for the shifted FP32/FP16 forms.
template <typename T>
struct Acc { using type = float; };
template <>
struct Acc<double> { using type = double; };
// Stored value s_i = f_i - shift_i, shift_i = w_i rho0 for the shifted forms
// and 0 for FP64; rest_i is the stored value of the rest state.
template <typename T>
constexpr bool kShifted = !std::is_same<T, double>::value;
template <bool SH, typename C>
__device__ inline C shift(int i, C rho0) {
  return SH ? wgt<C>(i) * rho0 : C(0);
}
template <bool SH, typename C>
__device__ inline C rest(int i, C rho0) {
  return SH ? C(0) : wgt<C>(i) * rho0;
}

// Element index of direction i of position q in a tiled population buffer
// ([np/kPopTile][19][kPopTile]).  Positions are below 2^30, so the tile
// arithmetic stays in 32 bits.
__device__ inline int64_t pidx(int32_t q, int i) {
  const int32_t row = (q >> kPopTileShift) * Q + i;
  return ((int64_t)row << kPopTileShift) + (int64_t)(q & (int32_t)(kPopTile - 1));
}

// Address of direction i of position q.  NARROW: the whole buffer is at most
// 4 GiB, so the byte offset is formed in 32 bits and the access takes the
// buffer's scalar base plus a 32-bit vector offset, which saves the 64-bit
// address arithmetic and the registers of 18 in-flight 64-bit addresses.
template <bool NARROW, typename T>
__device__ inline T *at(T *A, int32_t q, int i) {
  if constexpr (NARROW) {
    const uint32_t row = (uint32_t)((q >> kPopTileShift) * Q + i);
    const uint32_t e = (row << kPopTileShift) + (uint32_t)(q & (int32_t)(kPopTile - 1));
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T *>(reinterpret_cast<B *>(A) + e * (uint32_t)sizeof(T));
  } else {
    return A + pidx(q, i);
  }
}

// Cheaper addressing for the bulk+wall path of the step kernel when a buffer
// is at most 4 GiB.  Byte offset of (q, d) in a tiled buffer:
//   sz q + (q >> 12) KT + d D,   D = 4096 sz (one direction run of a tile),
//   KT = 18 D (the other runs of a tile).
// The direction term goes into a per-direction base held in scalar
// registers, dir_base(A, d) = A + d D - BIAS, and each lane supplies
//   voff(jb) = (jb >> (12 + log2 sz)) KT + jb,  jb = sz q + D,
// which equals sz q + (q >> 12) KT + BIAS (adding D = 2^(12 + log2 sz) to
// sz q adds exactly one to the tile number): one shift and one 24-bit
// multiply-add per address.  BIAS = KT + D keeps every lane offset
// non-negative, the reflected slot of a wall link included:
//   (p, opp(i)) = dir_base(A, i) + voff(sz p + D) + (opp(i) - i) D.
template <typename T>
struct Narrow {
  static constexpr uint32_t S = sizeof(T) == 8 ? 3u : (sizeof(T) == 4 ? 2u : 1u);
  static constexpr uint32_t D = uint32_t(kPopTile) * uint32_t(sizeof(T));
  static constexpr uint32_t KT = uint32_t(Q - 1) * D;
  static constexpr uint32_t BIAS = KT + D;
  static_assert(KT < (1u << 24), "24-bit multiply-add");
  __device__ static uint32_t voff(uint32_t jb) {
    return (jb >> (kPopTileShift + S)) * KT + jb;
  }
  // The empty asm keeps the compiler from folding the base's constant into
  // the lane offset (which would need 64-bit lane arithmetic): the load then
  // takes the scalar base plus the 32-bit lane offset.
  template <typename P>
  __device__ static P *at(P *A, int d, uint32_t off) {
    using GB = __attribute__((address_space(1))) char;
    GB *base = (GB *)A + (int64_t(d) * D - int64_t(BIAS));
    asm("" : "+s"(base));
    return (P *)(base + off);
  }
};

__device__ inline double ld(const double *p) { return *p; }
__device__ inline float ld(const float *p) { return *p; }
__device__ inline float ld(const _Float16 *p) { return static_cast<float>(*p); }
// Population stores and pull-table loads stream through HBM once per step:
// non-temporal, so that they do not displace the gathered lines from cache.
__device__ inline void st(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ inline void st(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ inline void st(_Float16 *p, float v) {
  __builtin_nontemporal_store(static_cast<_Float16>(v), p);  // round to nearest even
}
__device__ inline uint8_t ld_stream(const uint8_t *p) { return __builtin_nontemporal_load(p); }
// Cached stores, for the push scatter: its 64-element runs start anywhere, so
// neighbouring wavefronts complete each other's lines in L2 (non-temporal
// stores there measured 13-31% slower).
__device__ inline void st_cached(double *p, double v) { *p = v; }
__device__ inline void st_cached(float *p, float v) { *p = v; }
__device__ inline void st_cached(_Float16 *p, float v) { *p = static_cast<_Float16>(v); }

// Workgroups are dealt to the 8 XCDs round-robin by block id.  With a chunk
// size K > 0 the blocks are renumbered so that each XCD gets K consecutive
// tiles of every window of 8K tiles: neighbouring tiles then share that
// XCD's L2 while the chip as a whole still sweeps the site list in order.
// The last, partial window keeps the plain order.
__device__ inline int64_t block_id(int64_t b, int64_t G, int chunk) {
  if (chunk <= 0) return b;
  const int64_t win = 8 * (int64_t)chunk;
  const int64_t w = b / win;
  if ((w + 1) * win > G) return b;
  const int64_t r = b - w * win;
  return w * win + (r & 7) * chunk + (r >> 3);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-site outflow of a Windkessel outlet (k < 0: none), gathered while the
// site's links are processed; a site touching a second such outlet adds that
// one directly.
struct WkFlux {
  int k = -1;
  double q = 0.0;
  __device__ void add(double *acc, int kk, double v, int64_t stride = 1) {
    if (k < 0 || k == kk) {
      k = kk;
      q += v;
    } else {
      atomicAdd(acc + (int64_t)kk * stride, v);
    }
  }
};

// acc[k * stride] += the wavefront's summed q of every outlet k, one atomic
// per distinct k (the sites of one outlet are mostly neighbours in the iolet
// groups).  All 64 lanes must call it.
__device__ inline void wave_add_grouped(double *acc, const WkFlux &w, int64_t stride = 1) {
  bool pending = w.k >= 0;
  for (;;) {
    const uint64_t mask = __ballot(pending);
    if (mask == 0) break;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    const int kl = __shfl(w.k, leader, 64);
    const bool mine = pending && w.k == kl;
    const double s = wave_sum(mine ? w.q : 0.0);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(acc + (int64_t)kl * stride, s);
    if (mine) pending = false;
  }
}

// Moments (eqs. (5), (6)) of stored values s: rho = sum f, j = sum f c.
// Sums run in ascending i.  For the shifted forms rho = rho0 + sum s.
template <bool SH, typename C>
__device__ inline void moments(const C (&s)[Q], C rho0, C &dr, C &rho, C &jx, C &jy, C &jz) {
  dr = 0;
  jx = 0;
  jy = 0;
  jz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    dr += s[i];
    if (cx(i)) jx += cx(i) > 0 ? s[i] : -s[i];
    if (cy(i)) jy += cy(i) > 0 ? s[i] : -s[i];
    if (cz(i)) jz += cz(i) > 0 ? s[i] : -s[i];
  }
  rho = SH ? rho0 + dr : dr;
}

// Equilibrium eq. (4) (1/2 factors on the second-order terms) in the stored
// representation:  f_eq = w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u);
// shifted: f_eq - w rho0 = w (dr + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)) with
// dr = rho - rho0 passed in as summed, not recomputed from rho: in FP32,
// rho0 + dr rounds dr to the ulp of rho0, and that rounding would break the
// collision's mass conservation at every site and step.  dr is unused
// unshifted.
template <bool SH, typename C>
__device__ inline C s_eq(int i, C dr, C rho, C ux, C uy, C uz, C usq15) {
  const C cu = C(cx(i)) * ux + C(cy(i)) * uy + C(cz(i)) * uz;
  const C q = C(3) * cu + C(4.5) * cu * cu - usq15;
  return SH ? wgt<C>(i) * (dr + rho * q) : wgt<C>(i) * rho * (C(1) + q);
}

// BGK collision, eq. (3a) with dt = 1: s' = s + omega (s_eq - s).
template <bool SH, typename C>
__device__ inline void collide(C (&s)[Q], C omega, C rho0) {
  C dr, rho, jx, jy, jz;
  moments<SH>(s, rho0, dr, rho, jx, jy, jz);
  const C inv = C(1) / rho;
  const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int i = 0; i < Q; ++i) s[i] = s[i] + omega * (s_eq<SH>(i, dr, rho, ux, uy, uz, usq) - s[i]);
}

struct GatherArgs {
  const int32_t *seg_off;     // bulk+wall group: per-segment source offsets
  const int32_t *seg_base;
  const uint8_t *seg_delta;
  const int32_t *nbr_io;      // iolet groups: [18][nio] sources / link codes
  int64_t np;
  int64_t io_begin;
  int64_t nio;
  const double *corr;
  const IoletDev *io;
  const double *tables;
  const double *wk_rho;  // Windkessel outlet densities [n_iolets][2] by time parity
  double *io_flux;       // outflow accumulators of Windkessel outlets, or null (no accumulation)
  int64_t t;           // the update t -> t+1 uses the tables at t
  const int64_t *t_base;  // non-null inside a replayed graph: the time is *t_base + t
  const double *phi;   // porosity or null
  double rho0;
  int ladd_local;      // 1: the Ladd term takes the site's own density at t (else rho0)
};

// Time of the update an iolet rule belongs to (see GatherArgs::t_base).
__device__ inline int64_t step_time(const GatherArgs &a) { return a.t_base ? *a.t_base + a.t : a.t; }

static_assert(kBlock == kSegBlock, "one segment base per workgroup");
static_assert(kSegRow == 20, "segment rows are five 16-byte vectors");

// Source offsets of the 18 incoming links of bulk+wall position p, whose
// kSegBlock-position block is blk: off[i-1] = source - p, the source being
// a fluid position in [0, np), or for a wall link the offset np, which
// leaves [0, np) (the link then reads the site's own direction opp(i)).
__device__ inline void bulk_offsets(const GatherArgs &a, int64_t p, int64_t blk, int32_t (&off)[Q - 1]) {
  const int32_t s = a.seg_base[blk] + (int32_t)ld_stream(a.seg_delta + p);
  const int4 *row = reinterpret_cast<const int4 *>(a.seg_off + (int64_t)s * kSegRow);
  int4 r[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) r[k] = row[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off[4 * k] = r[k].x;
    off[4 * k + 1] = r[k].y;
    off[4 * k + 2] = r[k].z;
    off[4 * k + 3] = r[k].w;
  }
  off[16] = r[4].x;
  off[17] = r[4].y;
}

// bulk_offsets from p's row staged in LDS (the rows of p's block are the
// segments seg_base[blk] .. seg_base[blk] + seg_delta of its last position;
// p's row is entry seg_delta[p]).
__device__ inline void lds_offsets(const int4 *row, int32_t (&off)[Q - 1]) {
  int4 r[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) r[k] = row[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off[4 * k] = r[k].x;
    off[4 * k + 1] = r[k].y;
    off[4 * k + 2] = r[k].z;
    off[4 * k + 3] = r[k].w;
  }
  off[16] = r[4].x;
  off[17] = r[4].y;
}

// bulk_offsets for a whole wavefront (all 64 lanes active or not, each with
// its own p in ascending order): where the lanes' segments are at most two
// consecutive ones, both rows are read with scalar loads, which bypass the
// vector memory path's address processing, and each lane selects its row;
// otherwise every lane loads its own row.  The segment table carries one
// padding row, so that row first+1 exists.
__device__ inline void bulk_offsets_wave(const GatherArgs &a, int64_t p, int64_t blk, int32_t (&off)[Q - 1]) {
  const int32_t s = a.seg_base[blk] + (int32_t)ld_stream(a.seg_delta + p);
  const int32_t first = __builtin_amdgcn_readfirstlane(s);
  if (__ballot(s > first + 1) == 0) {
    using CI = const __attribute__((address_space(4))) int32_t;
    CI *r = (CI *)(a.seg_off + (int64_t)first * kSegRow);
    const bool second = s != first;
    // the empty asm statements hold both rows in scalar registers (else the
    // select folds into one per-lane load from a selected address)
#pragma unroll
    for (int i = 0; i < Q - 1; ++i) {
      int32_t x = r[i], y = r[kSegRow + i];
      asm("" : "+s"(x), "+s"(y));
      off[i] = second ? y : x;
    }
  } else {
    const int4 *row = reinterpret_cast<const int4 *>(a.seg_off + (int64_t)s * kSegRow);
    int4 rr[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) rr[k] = row[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      off[4 * k] = rr[k].x;
      off[4 * k + 1] = rr[k].y;
      off[4 * k + 2] = rr[k].z;
      off[4 * k + 3] = rr[k].w;
    }
    off[16] = rr[4].x;
    off[17] = rr[4].y;
  }
}

// Pre-collision populations of site p at time t+1, gathered from the
// post-collision buffer A of time t (stored values s = f - off), with the
// boundary rules (Sec. 2.3) for links that do not reach a fluid site:
//   wall (mid-link bounce-back):  f_i = f'_opp(i)(p); a porous wall site
//                                 returns (1 - phi) f'_opp(i) + phi w_i rho0
//   velocity iolet (Ladd):        f_i = f'_opp(i)(p) + 6 w_i rho0 (c_i.U(m)),
//                                 m = x - c_i/2, U = A_k(t) W(m) v_k
//   pressure iolet (ghost rho):   f_i = f_i^eq(rho_k(t), (u.n) n),
//                                 u the site's velocity at time t
// Returns the mass the boundary rules added (filled - reflected).  With
// a.io_flux set, the outflow of Windkessel outlets goes to *wkf (which must
// then be given).
// IOLET = false: the site has only fluid and wall links.
// blk: the kSegBlock-position block of p (bulk+wall group only).
// NARROW: see at().
// LROWS (bulk+wall group): p's segment row is staged in LDS at lrow (see
// lds_offsets).
template <bool IOLET, bool POROUS, bool SH, bool NARROW = false, bool LROWS = false, typename T, typename C>
__device__ inline C gather(const T *__restrict__ A, int64_t p, int64_t blk, const GatherArgs &a, C (&g)[Q],
                           WkFlux *wkf = nullptr, const int4 *lrow = nullptr) {
  const int64_t np = a.np;
  C flux = 0;
  if constexpr (!IOLET && NARROW) {
    // Bulk+wall group, buffers of at most 4 GiB (see Narrow).  A wall link's
    // offset np puts jb at or above sz np + D.
    using N = Narrow<T>;
    int32_t off[Q - 1];
    // FP16 is bound by the vector path's address processing: there the
    // scalar row loads took the step kernel from 0.335 to 0.330 ms on a
    // 2e7-site tree; FP64, bound by HBM, measured 0.2% slower with them.
    if constexpr (LROWS)
      lds_offsets(lrow, off);
    else if constexpr (sizeof(T) == 2)
      bulk_offsets_wave(a, p, blk, off);
    else
      bulk_offsets(a, p, blk, off);
    // The empty asm statements keep pb whole (so that each jb is one
    // shift-and-add) and make every lane compute its neighbour's offset (so
    // that the wall choice stays a select instead of a branch).
    uint32_t pb = ((uint32_t)p << N::S) + N::D;
    asm("" : "+v"(pb));
    const uint32_t own = N::voff(pb);
    const uint32_t wall_lo = own - N::D, wall_hi = own + N::D;  // (p, opp(i)) for even / odd i
    const uint32_t jb_wall = ((uint32_t)np << N::S) + N::D;
    g[0] = ld(N::at(A, 0, own));
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const uint32_t jb = ((uint32_t)off[i - 1] << N::S) + pb;
      uint32_t vj = N::voff(jb);
      asm("" : "+v"(vj));
      const bool wall = jb >= jb_wall;
      C v = ld(N::at(A, i, wall ? (opp(i) > i ? wall_hi : wall_lo) : vj));
      if constexpr (POROUS) {
        if (wall) {
          const C nv = v - C(a.phi[p]) * (v - rest<SH, C>(i, C(a.rho0)));
          flux += nv - v;
          v = nv;
        }
      }
      g[i] = v;
    }
  } else if constexpr (!IOLET) {
    // Bulk+wall group: every link, bounce-back included, is one load; the
    // offsets are fetched before the 18 gathers are issued.
    int32_t off[Q - 1];
    if constexpr (LROWS)
      lds_offsets(lrow, off);
    else
      bulk_offsets(a, p, blk, off);
    const int32_t p32 = (int32_t)p;
    g[0] = ld(at<NARROW>(A, p32, 0));
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      // a wall link's offset leaves [0, np): it reads the site's own
      // direction opp(i)
      const int32_t j = p32 + off[i - 1];
      const bool wall = (uint32_t)j >= (uint32_t)np;
      C v = ld(at<NARROW>(A, wall ? p32 : j, wall ? opp(i) : i));
      if constexpr (POROUS) {
        if (wall) {
          const C nv = v - C(a.phi[p]) * (v - rest<SH, C>(i, C(a.rho0)));
          flux += nv - v;
          v = nv;
        }
      }
      g[i] = v;
    }
  } else {
    // density and velocity at time t: moments of the site's own
    // post-collision state (the collision conserves rho and rho u)
    C ux, uy, uz, rho_x;
    {
      C own[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) own[i] = ld(at<NARROW>(A, (int32_t)p, i));
      C dr, jx, jy, jz;
      moments<SH>(own, C(a.rho0), dr, rho_x, jx, jy, jz);
      ux = jx / rho_x;
      uy = jy / rho_x;
      uz = jz / rho_x;
    }
    // the Ladd coefficients hold rho0; the local-density rule rescales them
    const double ladd_scale = a.ladd_local ? double(rho_x) / a.rho0 : 1.0;
    // The reflected values are read again below (cache hits) instead of
    // being kept live with the 19 gathered ones: the empty asm hides that
    // q == p, so the compiler cannot merge those reads with the ones above
    // and keep 19 more registers for them.
    const int64_t t = step_time(a);
    int32_t q = (int32_t)p;
    asm volatile("" : "+v"(q));
    g[0] = ld(at<NARROW>(A, q, 0));
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int32_t code = a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
      if (code >= 0) {
        g[i] = ld(at<NARROW>(A, code, i));
        continue;
      }
      const C back = ld(at<NARROW>(A, q, opp(i)));
      C v;
      if (code == HLB_LINK_WALL) {
        v = back;
        if constexpr (POROUS) v = back - C(a.phi[p]) * (back - rest<SH, C>(i, C(a.rho0)));
      } else {
        const int k = -code - 2;
        const IoletDev K = a.io[k];
        const double val = K.wk ? a.wk_rho[2 * k + (t & 1)] : a.tables[K.tab_off + t % K.tab_len];
        if (K.kind == HLB_IOLET_VELOCITY) {
          v = back + C(a.corr[(int64_t)(i - 1) * a.nio + (p - a.io_begin)] * val * ladd_scale);
        } else {
          const C un = ux * C(K.n[0]) + uy * C(K.n[1]) + uz * C(K.n[2]);
          const C gx = un * C(K.n[0]), gy = un * C(K.n[1]), gz = un * C(K.n[2]);
          const C uu = C(1.5) * (gx * gx + gy * gy + gz * gz);
          v = s_eq<SH>(i, C(val - a.rho0), C(val), gx, gy, gz, uu);
        }
        if (K.wk && a.io_flux) wkf->add(a.io_flux, k, double(back - v));
      }
      flux += v - back;
      g[i] = v;
    }
  }
  return flux;
}

// Two bulk+wall sites at once (gather<false, ...> for p and p2): both offset
// rows are fetched, then all 38 population loads are issued before any is
// used (the scheduling barrier keeps the compiler from interleaving the two
// sites' loads with the first site's arithmetic), so that a wavefront has
// twice the bytes in flight of the one-site form.  Returns the porous-wall
// flux of each site in flux1 / flux2.
template <bool POROUS, bool SH, bool NARROW, typename T, typename C>
__device__ inline void gather_bulk2(const T *__restrict__ A, int64_t p, int64_t blk, int64_t p2, int64_t blk2,
                                    const GatherArgs &a, C (&g)[Q], C (&h)[Q], C &flux1, C &flux2) {
  const int64_t np = a.np;
  int32_t o1[Q - 1], o2[Q - 1];
  bulk_offsets(a, p, blk, o1);
  bulk_offsets(a, p2, blk2, o2);
  const int32_t q1 = (int32_t)p, q2 = (int32_t)p2;
  uint32_t wall1 = 0, wall2 = 0;
  g[0] = ld(at<NARROW>(A, q1, 0));
  h[0] = ld(at<NARROW>(A, q2, 0));
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int32_t j1 = q1 + o1[i - 1], j2 = q2 + o2[i - 1];
    const bool w1 = (uint32_t)j1 >= (uint32_t)np, w2 = (uint32_t)j2 >= (uint32_t)np;
    g[i] = ld(at<NARROW>(A, w1 ? q1 : j1, w1 ? opp(i) : i));
    h[i] = ld(at<NARROW>(A, w2 ? q2 : j2, w2 ? opp(i) : i));
    if constexpr (POROUS) {
      wall1 |= (uint32_t)w1 << i;
      wall2 |= (uint32_t)w2 << i;
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  flux1 = 0;
  flux2 = 0;
  if constexpr (POROUS) {
    const C ph1 = C(a.phi[p]), ph2 = C(a.phi[p2]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if ((wall1 >> i) & 1u) {
        const C nv = g[i] - ph1 * (g[i] - rest<SH, C>(i, C(a.rho0)));
        flux1 += nv - g[i];
        g[i] = nv;
      }
      if ((wall2 >> i) & 1u) {
        const C nv = h[i] - ph2 * (h[i] - rest<SH, C>(i, C(a.rho0)));
        flux2 += nv - h[i];
        h[i] = nv;
      }
    }
  }
}

// Push order (the paper's implementation): site p has collided its own
// pre-collision state into fp (post-collision, stored representation); each
// population j goes where it arrives at t+1 -- slot j of the site at
// x + c_j, or, when that link leaves the fluid, the site's own slot opp(j)
// with the boundary rule's value (the rules of gather(), seen from the
// leaving side).  The site's link to x + c_j is the pull entry of direction
// opp(j), so the pull tables serve both orders.  (ux, uy, uz), rho_x: the
// site's velocity and density at t, for the pressure rule and the
// local-density Ladd rule.  Returns the mass the boundary rules
// added.
template <bool IOLET, bool POROUS, bool SH, bool NARROW, typename T, typename C>
__device__ inline C scatter(T *__restrict__ B, int64_t p, int64_t blk, const GatherArgs &a, const C (&fp)[Q], C ux,
                            C uy, C uz, C rho_x, WkFlux *wkf = nullptr) {
  const int64_t np = a.np;
  const int32_t p32 = (int32_t)p;
  C flux = 0;
  st_cached(at<NARROW>(B, p32, 0), fp[0]);
  if constexpr (!IOLET) {
    int32_t off[Q - 1];
    bulk_offsets(a, p, blk, off);
#pragma unroll
    for (int j = 1; j < Q; ++j) {
      const int32_t q = p32 + off[opp(j) - 1];
      const bool wall = (uint32_t)q >= (uint32_t)np;
      C v = fp[j];
      if constexpr (POROUS) {
        if (wall) {
          const C nv = v - C(a.phi[p]) * (v - rest<SH, C>(opp(j), C(a.rho0)));
          flux += nv - v;
          v = nv;
        }
      }
      st_cached(at<NARROW>(B, wall ? p32 : q, wall ? opp(j) : j), v);
    }
  } else {
    const int64_t t = step_time(a);
    const double ladd_scale = a.ladd_local ? double(rho_x) / a.rho0 : 1.0;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
      const int i = opp(j);  // the direction the boundary fills at p
      const int32_t code = a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
      if (code >= 0) {
        st_cached(at<NARROW>(B, code, j), fp[j]);
        continue;
      }
      const C back = fp[j];
      C v;
      if (code == HLB_LINK_WALL) {
        v = back;
        if constexpr (POROUS) v = back - C(a.phi[p]) * (back - rest<SH, C>(i, C(a.rho0)));
      } else {
        const int k = -code - 2;
        const IoletDev K = a.io[k];
        const double val = K.wk ? a.wk_rho[2 * k + (t & 1)] : a.tables[K.tab_off + t % K.tab_len];
        if (K.kind == HLB_IOLET_VELOCITY) {
          v = back + C(a.corr[(int64_t)(i - 1) * a.nio + (p - a.io_begin)] * val * ladd_scale);
        } else {
          const C un = ux * C(K.n[0]) + uy * C(K.n[1]) + uz * C(K.n[2]);
          const C gx = un * C(K.n[0]), gy = un * C(K.n[1]), gz = un * C(K.n[2]);
          const C uu = C(1.5) * (gx * gx + gy * gy + gz * gz);
          v = s_eq<SH>(i, C(val - a.rho0), C(val), gx, gy, gz, uu);
        }
        if (K.wk && a.io_flux) wkf->add(a.io_flux, k, double(back - v));
      }
      flux += v - back;
      st_cached(at<NARROW>(B, p32, i), v);
    }
  }
  return flux;
}

inline GatherArgs make_args(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int64_t t) {
  GatherArgs a;
  a.seg_off = d.seg_off;
  a.seg_base = d.seg_base;
  a.seg_delta = d.seg_delta;
  a.nbr_io = d.nbr_io;
  a.np = L.np;
  a.io_begin = L.io_begin;
  a.nio = L.nio;
  a.corr = d.corr;
  a.io = d.io;
  a.tables = d.tables;
  a.wk_rho = d.wk_rho;
  a.io_flux = d.io_flux;
  a.t = t;
  a.t_base = d.t_base;
  a.phi = cfg.porous ? d.phi : nullptr;
  a.rho0 = cfg.rho0;
  a.ladd_local = cfg.ladd_local ? 1 : 0;
  return a;
}

}  // namespace dev
}  // namespace hlb
