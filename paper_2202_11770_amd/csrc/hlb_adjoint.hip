// Adjoint (reverse-time) kernels of the pull update, FP64 storage.
//
// The paper defines no adjoint; this is the transpose of the update that
// hlb_kernels.hip computes.  With s_t the stored post-collision state at
// time t, g_t = G_t(s_{t-1}) the gathered pre-collision state (tables at
// t-1) and s_t = C(g_t) the BGK collision (eq. (3a), equilibrium eq. (4)),
// and the objective J = sum_{t in window} sum_x WSS(g_t(x)):
//   nu_t      = (dC/dg)^T mu_t + dJ_t/dg_t       (k_adj_collide, k_adj_boundary)
//   mu_{t-1}  = (dG_t/ds_{t-1})^T nu_t                      (k_adj_stream)
//   dJ/dA_k(t-1) = sum over Ladd links of nu_t,i corr_i
//   dJ/dphi_x   += sum over wall links of nu_t,i (rest_i - back_i)
// where mu_t = dJ/ds_t.  The transpose of the pull gather is again a gather
// (the site at x + c_i is the pull entry of direction opp(i)), so nothing is
// scattered and no further table is needed.

#include "hlb_adjoint.h"
#include "hlb_device.h"

namespace hlb {
namespace {

using namespace dev;

struct AdjArgs {
  GatherArgs a;             // forward gather arguments, tables at t-1
  const double *S;          // s_{t-1}: post-collision state at t-1 (tiled, as the state)
  double *mu;               // mu_t in, mu_{t-1} out (tiled)
  double *nu;               // nu_t (tiled)
  const int32_t *order;     // caller id per position (-1: padding)
  int64_t n0;               // sites of the bulk+wall group
  double omega, tau;
  int in_window;            // t lies in the objective window
  int64_t n_steps;          // row length of dA
  int64_t step;             // column of this step in dA: t-1-t0
  double *J;                // objective: [0] total, [8, 8 + kAdjJSlots) partial sums
  double *dA;               // [n_io][n_steps]: iolet table-value derivatives
  double *dphi;             // [np], accumulated over the sweep
  int objective;            // HLB_OBJ_WSS or HLB_OBJ_IOLET_FLUX
  const double *w;          // [n_io] iolet-flux weights of the objective
  // [n_io] outflow weights of this reverse step, dJ/dQ_k(t-1): the
  // objective's inside its window plus a Windkessel outlet's model term
  const double *wq;
};

// The value iolet k applies in the update a.t -> a.t+1: a Windkessel
// outlet's density from its model state, else the table value.
__device__ inline double iolet_value(const GatherArgs &a, const IoletDev &K, int k) {
  return K.wk ? a.wk_rho[2 * k + (a.t & 1)] : a.tables[K.tab_off + a.t % K.tab_len];
}

// The wavefront's share s of the objective, added to its partial-sum slot
// (one atomic per wavefront, spread over kAdjJSlots addresses); lane 0 adds.
__device__ inline void add_objective(double *J, double s) {
  static_assert((kAdjJSlots & (kAdjJSlots - 1)) == 0, "slot count is a power of two");
  if ((threadIdx.x & 63) == 0 && s != 0.0) {
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    atomicAdd(J + 8 + (wave & (kAdjJSlots - 1)), s);
  }
}

// (dM/dg)^T w for M(g) = f^eq(rho(g), u(g)):
//   sum_i w_i f^eq_i / rho + (sum_i w_i w8_i rho (3 c_i + 9 (c_i.u) c_i - 3 u)) . (c_j - u) / rho
// returned as the scalar a and the vector b with result_j = a + b.(c_j - u).
__device__ inline void eq_transpose(const double (&w)[Q], double rho, double ux, double uy, double uz,
                                    double &a, double &bx, double &by, double &bz) {
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
  a = 0.0;
  bx = by = bz = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    const double feq_over_rho = wgt<double>(i) * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq);
    a += w[i] * feq_over_rho;
    const double s = w[i] * wgt<double>(i);  // times rho, divided by rho
    bx += s * (3.0 * cx(i) + 9.0 * cu * cx(i) - 3.0 * ux);
    by += s * (3.0 * cy(i) + 9.0 * cu * cy(i) - 3.0 * uy);
    bz += s * (3.0 * cz(i) + 9.0 * cu * cz(i) - 3.0 * uz);
  }
}

// Link classes of position p in the pull tables: bit i-1 of `wall` is set
// when the entry of direction i is a wall link, of `iol` when it is an
// iolet link (the code is then read again where it is needed).
__device__ inline void link_masks(const GatherArgs &a, int64_t p, uint32_t &wall, uint32_t &iol) {
  wall = 0;
  iol = 0;
  if (p < a.io_begin) {
    int32_t off[Q - 1];
    bulk_offsets(a, p, p / kBlock, off);
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if ((uint32_t)((int32_t)p + off[i - 1]) >= (uint32_t)a.np) wall |= 1u << (i - 1);
  } else {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int32_t c = a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
      if (c == HLB_LINK_WALL) wall |= 1u << (i - 1);
      else if (c < HLB_LINK_WALL) iol |= 1u << (i - 1);
    }
  }
}

// The segment rows of a bulk+wall block staged in LDS, as in the forward
// step kernel (one coalesced pass instead of five row loads per lane, and
// per link-mask / gather pass): every thread of the block must call it.
// Returns p's row.
__device__ inline const int4 *stage_rows(const AdjArgs &A, int64_t blk, int64_t p, int4 *lrows) {
  const GatherArgs &a = A.a;
  const int32_t k_row = p < A.n0 ? (int32_t)ld_stream(a.seg_delta + p) : 0;
  const int64_t last = blk * kBlock + kBlock - 1 < A.n0 ? blk * kBlock + kBlock - 1 : A.n0 - 1;
  const int32_t n4 = ((int32_t)a.seg_delta[last] + 1) * (kSegRow / 4);
  const int4 *rows = reinterpret_cast<const int4 *>(a.seg_off + (int64_t)a.seg_base[blk] * kSegRow);
  for (int k = threadIdx.x; k < n4; k += kBlock) lrows[k] = rows[k];
  __syncthreads();
  return lrows + (kSegRow / 4) * k_row;
}

// link_masks of a bulk+wall position from its staged row.
__device__ inline uint32_t wall_mask(const GatherArgs &a, int64_t p, const int4 *lrow) {
  int32_t off[Q - 1];
  lds_offsets(lrow, off);
  uint32_t wall = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i)
    if ((uint32_t)((int32_t)p + off[i - 1]) >= (uint32_t)a.np) wall |= 1u << (i - 1);
  return wall;
}

// nu_t = (dC/dg)^T mu_t + dWSS/dg_t for every site (the parameter terms
// follow in k_adj_boundary, at the sites that have them).  The gathered
// state g lives only until its moments are known.  mu is read once and nu
// written once per step, both far beyond the caches: non-temporal (measured
// 12% off the reverse step with the same in k_adj_stream).
//
// Without porosity the porosity derivative is taken here too: at a wall link
// j the gathered value is g_j = s_{t-1}(p, opp(j)), so with h_j = w_j rho0 -
// g_j and nu_j = (1 - omega) mu_j + omega (a + b.(c_j - u)) + d_j (d: the
// WSS term below),
//   sum over wall links of nu_j h_j
//     = (1 - omega) sum mu_j h_j + omega (a H + b.(Hc - u H)) + sum d_j h_j,
//   H = sum h_j,  Hc = sum h_j c_j.
// Outside the WSS window mu is loaded with the gather, so that sum mu_j h_j
// is formed before g is dropped.  This spares k_adj_boundary the scattered
// loads of nu and s_{t-1} at every wall site.  With porosity the gathered
// value is not s_{t-1} itself, and k_adj_boundary keeps the whole term.
//
// WSS (the WSS objective inside its window): J += WSS(g_t) and its
// gradient.  With n the wall normal, s the tangential traction, fac =
// -(1 - 1/(2 tau)) and e = s/|s|, the stress is fac (sum g c c - sum f^eq c
// c), sum f^eq c c = rho/3 I + rho u u (eq. (4) with the 1/2 factors), so
//   d_j = dWSS/dg_j = fac e.(c_j c_j - I/3 - c_j u - u c_j + u u) n
//       = ((c_j - u).n)((c_j - u).E),   E = fac e   (e.n = 0).
// Only the six second moments of g are formed while g is live, and the
// traction is reduced to n and E before mu is loaded; h_j then re-reads the
// site's own slot s_{t-1}(p, opp(j)) at its wall links.
template <bool POROUS, bool WSS>
__global__ __launch_bounds__(kBlock) void k_adj_collide(AdjArgs A) {
  const GatherArgs &a = A.a;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  // bulk+wall blocks (block-uniform): the segment rows through LDS
  __shared__ int4 lrows[kSegBlock * (kSegRow / 4)];
  const bool bulk = (int64_t)blockIdx.x * kBlock < A.n0;
  const int4 *lrow = bulk ? stage_rows(A, blockIdx.x, p, lrows) : nullptr;
  double jsum = 0.0;
  if (p < a.np && A.order[p] >= 0) {
    const int32_t p32 = (int32_t)p;
    double rho, ux, uy, uz;
    double m[Q];
    double hm = 0.0, h0 = 0.0, hx = 0.0, hy = 0.0, hz = 0.0;
    double pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;  // second moments of g
    uint32_t wall = 0;
    if constexpr (!POROUS || WSS) {
      if (bulk) {
        wall = wall_mask(a, p, lrow);
      } else {
        uint32_t iol;
        link_masks(a, p, wall, iol);
      }
    }
    constexpr bool kMuEarly = !POROUS && !WSS;
    {
      double g[Q];
      if (bulk)
        gather<false, POROUS, false, false, true>(A.S, p, p / kBlock, a, g, nullptr, lrow);
      else
        gather<true, POROUS, false>(A.S, p, 0, a, g);
      if constexpr (kMuEarly) {
#pragma unroll
        for (int i = 0; i < Q; ++i) m[i] = __builtin_nontemporal_load(&A.mu[pidx(p32, i)]);
      }
      double dr, jx, jy, jz;
      moments<false>(g, 0.0, dr, rho, jx, jy, jz);
      ux = jx / rho;
      uy = jy / rho;
      uz = jz / rho;
      if constexpr (WSS) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          if (cx(i)) pxx += g[i];
          if (cy(i)) pyy += g[i];
          if (cz(i)) pzz += g[i];
          if (cx(i) && cy(i)) pxy += cx(i) * cy(i) > 0 ? g[i] : -g[i];
          if (cx(i) && cz(i)) pxz += cx(i) * cz(i) > 0 ? g[i] : -g[i];
          if (cy(i) && cz(i)) pyz += cy(i) * cz(i) > 0 ? g[i] : -g[i];
        }
      }
      if constexpr (kMuEarly) {
#pragma unroll
        for (int j = 1; j < Q; ++j) {
          const double h = ((wall >> (j - 1)) & 1u) ? wgt<double>(j) * a.rho0 - g[j] : 0.0;
          hm += m[j] * h;
          h0 += h;
          hx += h * cx(j);
          hy += h * cy(j);
          hz += h * cz(j);
        }
      }
    }
    // the WSS term's n and E (zero without a wall normal or traction)
    double nx = 0, ny = 0, nz = 0, Ex = 0, Ey = 0, Ez = 0;
    if constexpr (WSS) {
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (wall & (1u << (i - 1))) {
          nx -= cx(i);
          ny -= cy(i);
          nz -= cz(i);
        }
      const double nn = sqrt(nx * nx + ny * ny + nz * nz);
      if (nn > 0.0) {
        nx /= nn;
        ny /= nn;
        nz /= nn;
        const double fac = -(1.0 - 1.0 / (2.0 * A.tau));
        pxx -= rho * (1.0 / 3.0 + ux * ux);
        pyy -= rho * (1.0 / 3.0 + uy * uy);
        pzz -= rho * (1.0 / 3.0 + uz * uz);
        pxy -= rho * ux * uy;
        pxz -= rho * ux * uz;
        pyz -= rho * uy * uz;
        const double tx = fac * (pxx * nx + pxy * ny + pxz * nz);
        const double ty = fac * (pxy * nx + pyy * ny + pyz * nz);
        const double tz = fac * (pxz * nx + pyz * ny + pzz * nz);
        const double tn = tx * nx + ty * ny + tz * nz;
        const double sx = tx - tn * nx, sy = ty - tn * ny, sz = tz - tn * nz;
        const double w = sqrt(sx * sx + sy * sy + sz * sz);
        jsum = w;
        if (w > 0.0) {
          const double fw = fac / w;
          Ex = fw * sx;
          Ey = fw * sy;
          Ez = fw * sz;
        } else {
          nx = ny = nz = 0.0;
        }
      }
      // g is consumed: the loads below start after these are formed
      asm volatile("" ::"v"(rho), "v"(ux), "v"(uy), "v"(uz), "v"(nx), "v"(ny), "v"(nz), "v"(Ex), "v"(Ey), "v"(Ez)
                   : "memory");
    }
    const double un = ux * nx + uy * ny + uz * nz, uE = ux * Ex + uy * Ey + uz * Ez;
    if constexpr (!kMuEarly) {
#pragma unroll
      for (int i = 0; i < Q; ++i) m[i] = __builtin_nontemporal_load(&A.mu[pidx(p32, i)]);
    }
    double dphi = 0.0;
    if constexpr (!POROUS && WSS) {
      if (wall) {
#pragma unroll
        for (int j = 1; j < Q; ++j) {
          if (!((wall >> (j - 1)) & 1u)) continue;
          const double h = wgt<double>(j) * a.rho0 - A.S[pidx(p32, opp(j))];
          hm += m[j] * h;
          h0 += h;
          hx += h * cx(j);
          hy += h * cy(j);
          hz += h * cz(j);
          dphi += h * (cx(j) * nx + cy(j) * ny + cz(j) * nz - un) * (cx(j) * Ex + cy(j) * Ey + cz(j) * Ez - uE);
        }
      }
    }
    double ea, ebx, eby, ebz;
    eq_transpose(m, rho, ux, uy, uz, ea, ebx, eby, ebz);
    if constexpr (!POROUS) {
      if (wall)
        A.dphi[p] += dphi + (1.0 - A.omega) * hm +
                     A.omega * (ea * h0 + ebx * (hx - ux * h0) + eby * (hy - uy * h0) + ebz * (hz - uz * h0));
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      double v = (1.0 - A.omega) * m[j] + A.omega * (ea + ebx * (cx(j) - ux) + eby * (cy(j) - uy) + ebz * (cz(j) - uz));
      if constexpr (WSS) v += (cx(j) * nx + cy(j) * ny + cz(j) * nz - un) * (cx(j) * Ex + cy(j) * Ey + cz(j) * Ez - uE);
      __builtin_nontemporal_store(v, &A.nu[pidx(p32, j)]);
    }
  }
  if constexpr (WSS) add_objective(A.J, wave_sum(jsum));
}

// The parameter derivatives of the update t-1 -> t, and the iolet-flux
// objective, at the sites with wall or iolet links (list, ascending
// positions); nu_t is complete when this runs:
//   porosity: dJ/dphi_x += sum over wall links of nu_i (rest_i - back_i)
//     (without porosity k_adj_collide takes the whole term, so the kernel
//     then runs over the sites with iolet links alone);
//   iolet table values: dJ/dA_k(t-1) += sum over links of k of (nu_i - w_k)
//     d(fill_i)/dA_k, w_k = dJ/dQ_k(t-1) the step's outflow weight, and with
//     the iolet-flux objective J += (its weight) (leaving population - fill)
//     per link.
// It loads nu only at the site's wall and iolet links.  Compiled for 2
// waves per SIMD: measured 2% faster per reverse step than the compiler's
// default (4 waves) and than 1 or 3.
template <bool POROUS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adj_boundary(
    AdjArgs A, const int32_t *__restrict__ list, int64_t n_list) {
  const GatherArgs &a = A.a;
  const int64_t k_site = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double jsum = 0.0;
  WkFlux dtab;  // this site's table-value derivative (one iolet per site, mostly)
  if (k_site < n_list) {
    const int64_t p = list[k_site];
    const int32_t p32 = (int32_t)p;
    uint32_t wall, iol;
    link_masks(a, p, wall, iol);
    // nu of this site's wall and iolet links (bit i: direction i)
    const uint32_t need = ((POROUS ? wall : 0u) | iol) << 1;
    double m[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) m[i] = ((need >> i) & 1u) ? A.nu[pidx(p32, i)] : 0.0;
    if constexpr (POROUS) {
      double dphi = 0.0;
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (wall & (1u << (i - 1))) dphi += m[i] * (wgt<double>(i) * a.rho0 - A.S[pidx(p32, opp(i))]);
      if (dphi != 0.0) A.dphi[p] += dphi;
    }
    if (iol) {
      const bool flux = A.objective == HLB_OBJ_IOLET_FLUX && A.in_window;
      double ox, oy, oz;  // velocity at t-1 (pressure rule)
      {
        double s[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) s[i] = A.S[pidx(p32, i)];
        double sdr, srho, sjx, sjy, sjz;
        moments<false>(s, 0.0, sdr, srho, sjx, sjy, sjz);
        ox = sjx / srho;
        oy = sjy / srho;
        oz = sjz / srho;
      }
      double q = 0.0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        if (!(iol & (1u << (i - 1)))) continue;
        const int k = -a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)] - 2;
        const IoletDev K = a.io[k];
        const double val = iolet_value(a, K, k);
        const double wk = A.wq[k];
        const double wo = flux ? A.w[k] : 0.0;
        double coef, out;  // d(filled value)/d(table value); outflow of the link
        if (K.kind == HLB_IOLET_VELOCITY) {
          coef = a.corr[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
          out = -coef * val;
        } else {
          const double un = ox * K.n[0] + oy * K.n[1] + oz * K.n[2];
          const double gx = un * K.n[0], gy = un * K.n[1], gz = un * K.n[2];
          coef = s_eq<false>(i, 0.0, 1.0, gx, gy, gz, 1.5 * (gx * gx + gy * gy + gz * gz));
          out = A.S[pidx(p32, opp(i))] - val * coef;
        }
        dtab.add(A.dA + A.step, k, (m[i] - wk) * coef, A.n_steps);
        q += wo * out;
      }
      if (flux) jsum = q;
    }
  }
  add_objective(A.J, wave_sum(jsum));
  wave_add_grouped(A.dA + A.step, dtab, A.n_steps);  // one atomic per iolet per wavefront
}

// mu_{t-1} = (dG_t/ds_{t-1})^T nu_t (compiled for 4 waves per SIMD; only the
// iolet path spills, and the default allocation gave 3): population i of p at t-1 went to the
// site at x + c_i -- the pull entry of direction opp(i), which names the
// site that pulled it --, was reflected back to p (wall: times 1 - phi;
// Ladd: plus a constant), or was replaced (pressure iolet: no direct path,
// but the fill depends on p's velocity at t-1).
template <bool POROUS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_adj_stream(AdjArgs A) {
  const GatherArgs &a = A.a;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  // bulk+wall blocks (block-uniform): the segment rows through LDS
  __shared__ int4 lrows[kSegBlock * (kSegRow / 4)];
  const bool bulk = (int64_t)blockIdx.x * kBlock < A.n0;
  const int4 *lrow = bulk ? stage_rows(A, blockIdx.x, p, lrows) : nullptr;
  if (p >= a.np || A.order[p] < 0) return;
  const int32_t p32 = (int32_t)p;
  const double ph = POROUS ? a.phi[p] : 0.0;
  // outflow weights w_k = dJ/dQ_k(t-1): a population leaving through a
  // pressure iolet adds w_k to its own adjoint (the fill does not depend on
  // it), and the fill's dependence on u enters with weight (nu - w_k)
  if (bulk) {
    // bulk+wall group (block-uniform): fluid and wall links only, one load
    // per link as in the forward gather
    // All 19 loads are issued before the first store: mu and nu are
    // different buffers, but the compiler cannot know it, and a store
    // between two loads would make each load wait for the one before.
    int32_t off[Q - 1];
    lds_offsets(lrow, off);
    double v[Q];
    v[0] = A.nu[pidx(p32, 0)];
    uint32_t walls = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int32_t q = p32 + off[opp(i) - 1];
      const bool wall = (uint32_t)q >= (uint32_t)a.np;
      v[i] = A.nu[pidx(wall ? p32 : q, wall ? opp(i) : i)];
      if (POROUS) walls |= (uint32_t)wall << i;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store((POROUS && ((walls >> i) & 1u)) ? (1.0 - ph) * v[i] : v[i], &A.mu[pidx(p32, i)]);
    return;
  }
  // iolet groups: the site's 18 pull entries
  int32_t code[Q - 1];
#pragma unroll
  for (int i = 1; i < Q; ++i) code[i - 1] = a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
  double m[Q];
  bool pressure = false;
  m[0] = A.nu[pidx(p32, 0)];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int32_t c = code[opp(i) - 1];
    if (c >= 0) {
      m[i] = A.nu[pidx(c, i)];
    } else if (c == HLB_LINK_WALL) {
      m[i] = (1.0 - ph) * A.nu[pidx(p32, opp(i))];
    } else if (a.io[-c - 2].kind == HLB_IOLET_VELOCITY) {
      m[i] = A.nu[pidx(p32, opp(i))];
    } else {
      m[i] = A.wq[-c - 2];  // replaced by the ghost-density equilibrium
      pressure = true;
    }
  }
  if (pressure) {
    // the ghost equilibrium depends on the site's u at t-1 (moments of s_{t-1})
    double s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = A.S[pidx(p32, i)];
    double dr, rho, jx, jy, jz;
    moments<false>(s, 0.0, dr, rho, jx, jy, jz);
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int32_t c = code[opp(i) - 1];
      if (c >= HLB_LINK_WALL) continue;
      const IoletDev K = a.io[-c - 2];
      if (K.kind != HLB_IOLET_PRESSURE) continue;
      const int o = opp(i);  // incoming population = f^eq_o(rho_k, (u.n) n)
      const double rk = iolet_value(a, K, -c - 2);
      const double un = ux * K.n[0] + uy * K.n[1] + uz * K.n[2];
      const double gx = un * K.n[0], gy = un * K.n[1], gz = un * K.n[2];
      const double cu = cx(o) * gx + cy(o) * gy + cz(o) * gz;
      const double dx = wgt<double>(o) * rk * (3.0 * cx(o) + 9.0 * cu * cx(o) - 3.0 * gx);
      const double dy = wgt<double>(o) * rk * (3.0 * cy(o) + 9.0 * cu * cy(o) - 3.0 * gy);
      const double dz = wgt<double>(o) * rk * (3.0 * cz(o) + 9.0 * cu * cz(o) - 3.0 * gz);
      const double wk = A.wq[-c - 2];
      const double coef = (A.nu[pidx(p32, o)] - wk) * (dx * K.n[0] + dy * K.n[1] + dz * K.n[2]) / rho;
#pragma unroll
      for (int j = 0; j < Q; ++j)
        m[j] += coef * (K.n[0] * (cx(j) - ux) + K.n[1] * (cy(j) - uy) + K.n[2] * (cz(j) - uz));
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(m[i], &A.mu[pidx(p32, i)]);
}

// Outflow weights of the reverse step of the update s -> s+1 (s = step):
// the objective's weight inside its window, plus, for a Windkessel outlet,
// dJ/dQ_k(s) from the adjoint of its model (R19 of the readings):
//   LX(s+1) = Lr(s+1) + kappa LX(s+2),  kappa = dX(s+2)/dX(s+1),
//   dJ/dQ_k(s) = R1 Lr(s+1) + dX(s+1)/dQ LX(s+1),
// Lr(s+1) = column s+1 of dA (the derivative with respect to the density of
// step s+1, written by the previous reverse step), zero past the last step.
// lamX holds LX(s+2) on entry and LX(s+1) on return.
__global__ void k_adj_weights(const IoletDev *io, const WkParams *wk, int n_io, const double *dA,
                              int64_t n_steps, int64_t step, const double *w, int flux, double *lamX,
                              double *wq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_io) return;
  double v = flux ? w[k] : 0.0;
  if (wk && io[k].wk) {
    const WkParams P = wk[k];
    const double lr = step + 1 < n_steps ? dA[(int64_t)k * n_steps + step + 1] : 0.0;
    const double kappa = P.C > 0.0 ? 1.0 - (P.R2 > 0.0 ? 1.0 / (P.R2 * P.C) : 0.0) : 0.0;
    const double lx = lr + kappa * lamX[k];
    v += P.R1 * lr + (P.C > 0.0 ? 1.0 / P.C : P.R2) * lx;
    lamX[k] = lx;
  }
  wq[k] = v;
}

// J[0] := sum of the kAdjJSlots partial sums (one workgroup of kBlock).
__global__ __launch_bounds__(kBlock) void k_adj_objective(double *J) {
  __shared__ double part[kBlock / 64];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < kAdjJSlots; i += kBlock) v += J[8 + i];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += part[w];
    J[0] = t;
  }
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_adjoint_step(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src, int64_t t,
                               const AdjBuffers &b, int in_window, int64_t n_steps, int64_t step,
                               hipStream_t s) {
  if (cfg.storage != HLB_F64) return hipErrorInvalidValue;
  AdjArgs A;
  A.a = make_args(cfg, L, d, t - 1);
  A.a.io_flux = nullptr;
  A.S = static_cast<const double *>(d.f[src]);
  A.mu = b.mu;
  A.nu = b.nu;
  A.order = d.order;
  A.n0 = L.gcnt[0];
  A.omega = 1.0 / cfg.tau;
  A.tau = cfg.tau;
  A.in_window = in_window;
  A.n_steps = n_steps;
  A.step = step;
  A.J = b.J;
  A.dA = b.dA;
  A.dphi = b.dphi;
  A.objective = b.objective;
  A.w = b.w;
  A.wq = b.wq;
  if (b.n_io > 0) {
    if (!b.wq || !b.lamX) return hipErrorInvalidValue;
    k_adj_weights<<<(b.n_io + 63) / 64, 64, 0, s>>>(d.io, d.wk, b.n_io, b.dA, n_steps, step, b.w,
                                                    b.objective == HLB_OBJ_IOLET_FLUX && in_window, b.lamX, b.wq);
  }
  const bool wss = b.objective == HLB_OBJ_WSS && in_window;
  const unsigned grid = blocks_of(L.np);
  if (cfg.porous) {
    if (wss)
      k_adj_collide<true, true><<<grid, kBlock, 0, s>>>(A);
    else
      k_adj_collide<true, false><<<grid, kBlock, 0, s>>>(A);
    if (b.n_blist > 0)
      k_adj_boundary<true><<<blocks_of(b.n_blist), kBlock, 0, s>>>(A, b.blist, b.n_blist);
    k_adj_stream<true><<<grid, kBlock, 0, s>>>(A);
  } else {
    if (wss)
      k_adj_collide<false, true><<<grid, kBlock, 0, s>>>(A);
    else
      k_adj_collide<false, false><<<grid, kBlock, 0, s>>>(A);
    // without porosity only the sites with iolet links (the list's tail)
    // have terms left
    const int64_t n_list = b.n_blist - b.n_blist_wall;
    if (n_list > 0) k_adj_boundary<false><<<blocks_of(n_list), kBlock, 0, s>>>(A, b.blist + b.n_blist_wall, n_list);
    k_adj_stream<false><<<grid, kBlock, 0, s>>>(A);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_objective(double *J, hipStream_t s) {
  k_adj_objective<<<1, kBlock, 0, s>>>(J);
  return hipGetLastError();
}

}  // namespace hlb
