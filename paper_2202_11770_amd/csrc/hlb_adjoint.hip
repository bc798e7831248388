// Adjoint (reverse-time) kernels of the pull update, FP64 storage.
//
// The paper defines no adjoint; this is the transpose of the update that
// hlb_kernels.hip computes.  With s_t the stored post-collision state at
// time t, g_t = G_t(s_{t-1}) the gathered pre-collision state (tables at
// t-1) and s_t = C(g_t) the BGK collision (eq. (3a), equilibrium eq. (4)),
// and the objective J = sum_{t in window} sum_x WSS(g_t(x)):
//   nu_t      = (dC/dg)^T mu_t + dJ_t/dg_t                 (k_adj_collide)
//   mu_{t-1}  = (dG_t/ds_{t-1})^T nu_t                      (k_adj_stream)
//   dJ/dA_k(t-1) = sum over Ladd links of nu_t,i corr_i
//   dJ/dphi_x   += sum over wall links of nu_t,i (rest_i - back_i)
// where mu_t = dJ/ds_t.  The transpose of the pull gather is again a gather,
// through the push table (the position of x + c_i), so nothing is scattered.

#include "hlb_device.h"

namespace hlb {
namespace {

using namespace dev;

struct AdjArgs {
  GatherArgs a;             // forward gather arguments, tables at t-1
  const double *S;          // s_{t-1}: post-collision state at t-1 (tiled, as the state)
  double *mu;               // mu_t in, mu_{t-1} out (tiled)
  double *nu;               // nu_t (tiled)
  const int32_t *push;      // [18][np]: position of x + c_i, or the link code
  const int32_t *order;     // caller id per position (-1: padding)
  double omega, tau;
  int in_window;            // t lies in the objective window
  int64_t n_steps;          // row length of dA
  int64_t step;             // column of this step in dA: t-1-t0
  double *J;                // objective accumulator
  double *dA;               // [n_io][n_steps]: iolet table-value derivatives
  double *dphi;             // [np], accumulated over the sweep
  int objective;            // HLB_OBJ_WSS or HLB_OBJ_IOLET_FLUX
  const double *w;          // [n_io] iolet-flux weights
};

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

template <bool POROUS>
__global__ __launch_bounds__(kBlock) void k_adj_collide(AdjArgs A) {
  const GatherArgs &a = A.a;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double jsum = 0.0;
  if (p < a.np && A.order[p] >= 0) {
    const bool bulk = p < a.io_begin;
    double g[Q];
    if (bulk)
      gather<false, POROUS, false>(A.S, p, p / kBlock, a, g);
    else
      gather<true, POROUS, false>(A.S, p, 0, a, g);
    double dr, rho, jx, jy, jz;
    moments<false>(g, 0.0, dr, rho, jx, jy, jz);
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    double m[Q], nu[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) m[i] = A.mu[pidx((int32_t)p, i)];
    double ea, ebx, eby, ebz;
    eq_transpose(m, rho, ux, uy, uz, ea, ebx, eby, ebz);
#pragma unroll
    for (int j = 0; j < Q; ++j)
      nu[j] = (1.0 - A.omega) * m[j] + A.omega * (ea + ebx * (cx(j) - ux) + eby * (cy(j) - uy) + ebz * (cz(j) - uz));
    // link codes of the site (-1 wall, -(2+k) iolet k, >= 0 fluid) and the
    // wall-link normal
    int32_t code[Q - 1];
    int32_t off[Q - 1];
    if (bulk) bulk_offsets(a, p, p / kBlock, off);
    double nx = 0, ny = 0, nz = 0;
    bool any = false;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (bulk)
        code[i - 1] = (uint64_t)(p + (int64_t)off[i - 1]) >= (uint64_t)a.np ? HLB_LINK_WALL : 0;
      else
        code[i - 1] = a.nbr_io[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
      if (code[i - 1] == HLB_LINK_WALL) {
        any = true;
        nx -= cx(i);
        ny -= cy(i);
        nz -= cz(i);
      }
    }
    // objective: wall shear stress of g and its gradient (definition of k_macros)
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    if (A.objective == HLB_OBJ_WSS && A.in_window && any && nn > 0.0) {
      nx /= nn;
      ny /= nn;
      nz /= nn;
      const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
      double pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double d = g[i] - s_eq<false>(i, 0.0, rho, ux, uy, uz, usq);
        pxx += d * cx(i) * cx(i);
        pyy += d * cy(i) * cy(i);
        pzz += d * cz(i) * cz(i);
        pxy += d * cx(i) * cy(i);
        pxz += d * cx(i) * cz(i);
        pyz += d * cy(i) * cz(i);
      }
      const double fac = -(1.0 - 1.0 / (2.0 * A.tau));
      const double tx = fac * (pxx * nx + pxy * ny + pxz * nz);
      const double ty = fac * (pxy * nx + pyy * ny + pyz * nz);
      const double tz = fac * (pxz * nx + pyz * ny + pzz * nz);
      const double tn = tx * nx + ty * ny + tz * nz;
      const double sx = tx - tn * nx, sy = ty - tn * ny, sz = tz - tn * nz;
      const double w = sqrt(sx * sx + sy * sy + sz * sz);
      jsum = w;
      if (w > 0.0) {
        // dWSS/d(g - f^eq)_i = fac (c_i.n)(e.c_i), e = s/|s|; then through f^eq(g)
        double wd[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
          wd[i] = fac * (cx(i) * nx + cy(i) * ny + cz(i) * nz) * (cx(i) * sx + cy(i) * sy + cz(i) * sz) / w;
        double wa, wbx, wby, wbz;
        eq_transpose(wd, rho, ux, uy, uz, wa, wbx, wby, wbz);
#pragma unroll
        for (int j = 0; j < Q; ++j)
          nu[j] += wd[j] - (wa + wbx * (cx(j) - ux) + wby * (cy(j) - uy) + wbz * (cz(j) - uz));
      }
    }
    // parameter derivatives from the complete nu_t: porosity at wall links,
    // the table value (amplitude or ghost density) at iolet links.  With the
    // iolet-flux objective the update t-1 -> t adds, per iolet link,
    // w_k (leaving population - filled value) to J, and -w_k times the
    // filled value's table derivative to that derivative.
    const bool flux = A.objective == HLB_OBJ_IOLET_FLUX && A.in_window;
    double ox = 0.0, oy = 0.0, oz = 0.0;  // velocity at t-1 (pressure rule)
    if (!bulk) {
      double s[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) s[i] = A.S[pidx((int32_t)p, i)];
      double sdr, srho, sjx, sjy, sjz;
      moments<false>(s, 0.0, sdr, srho, sjx, sjy, sjz);
      ox = sjx / srho;
      oy = sjy / srho;
      oz = sjz / srho;
    }
    double dphi = 0.0, q = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int32_t c = code[i - 1];
      if (c == HLB_LINK_WALL) {
        const double back = A.S[pidx((int32_t)p, opp(i))];
        dphi += nu[i] * (wgt<double>(i) * a.rho0 - back);
      } else if (c < HLB_LINK_WALL) {
        const int k = -c - 2;
        const IoletDev K = a.io[k];
        const double val = a.tables[K.tab_off + a.t % K.tab_len];
        const double wk = flux ? A.w[k] : 0.0;
        double coef, out;  // d(filled value)/d(table value); outflow of the link
        if (K.kind == HLB_IOLET_VELOCITY) {
          coef = a.corr[(int64_t)(i - 1) * a.nio + (p - a.io_begin)];
          out = -coef * val;
        } else {
          const double un = ox * K.n[0] + oy * K.n[1] + oz * K.n[2];
          const double gx = un * K.n[0], gy = un * K.n[1], gz = un * K.n[2];
          coef = s_eq<false>(i, 0.0, 1.0, gx, gy, gz, 1.5 * (gx * gx + gy * gy + gz * gz));
          out = A.S[pidx((int32_t)p, opp(i))] - val * coef;
        }
        atomicAdd(A.dA + (int64_t)k * A.n_steps + A.step, (nu[i] - wk) * coef);
        q += wk * out;
      }
    }
    if (flux) jsum = q;
    A.dphi[p] += dphi;
#pragma unroll
    for (int i = 0; i < Q; ++i) A.nu[pidx((int32_t)p, i)] = nu[i];
  }
  const double s = wave_sum(jsum);
  if ((threadIdx.x & 63) == 0 && s != 0.0) atomicAdd(A.J, s);
}

template <bool POROUS>
__global__ __launch_bounds__(kBlock) void k_adj_stream(AdjArgs A) {
  const GatherArgs &a = A.a;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= a.np || A.order[p] < 0) return;
  const double ph = POROUS ? a.phi[p] : 0.0;
  // iolet-flux objective: a population leaving through a pressure iolet adds
  // w_k to its own adjoint (the fill does not depend on it), and the fill's
  // dependence on u enters with weight (nu - w_k)
  const bool flux = A.objective == HLB_OBJ_IOLET_FLUX && A.in_window;
  double m[Q];
  bool pressure = false;
  m[0] = A.nu[pidx((int32_t)p, 0)];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    // s_{t-1}[i][p] was read by the site at p + c_i, or reflected back to p
    const int32_t c = A.push[(int64_t)(i - 1) * a.np + p];
    if (c >= 0) {
      m[i] = A.nu[pidx((int32_t)c, i)];
    } else if (c == HLB_LINK_WALL) {
      m[i] = (1.0 - ph) * A.nu[pidx((int32_t)p, opp(i))];
    } else if (a.io[-c - 2].kind == HLB_IOLET_VELOCITY) {
      m[i] = A.nu[pidx((int32_t)p, opp(i))];
    } else {
      m[i] = flux ? A.w[-c - 2] : 0.0;  // replaced by the ghost-density equilibrium
      pressure = true;
    }
  }
  if (pressure) {
    // the ghost equilibrium depends on the site's u at t-1 (moments of s_{t-1})
    double s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = A.S[pidx((int32_t)p, i)];
    double dr, rho, jx, jy, jz;
    moments<false>(s, 0.0, dr, rho, jx, jy, jz);
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int32_t c = A.push[(int64_t)(i - 1) * a.np + p];
      if (c >= HLB_LINK_WALL) continue;
      const IoletDev K = a.io[-c - 2];
      if (K.kind != HLB_IOLET_PRESSURE) continue;
      const int o = opp(i);  // incoming population = f^eq_o(rho_k, (u.n) n)
      const double rk = a.tables[K.tab_off + a.t % K.tab_len];
      const double un = ux * K.n[0] + uy * K.n[1] + uz * K.n[2];
      const double gx = un * K.n[0], gy = un * K.n[1], gz = un * K.n[2];
      const double cu = cx(o) * gx + cy(o) * gy + cz(o) * gz;
      const double dx = wgt<double>(o) * rk * (3.0 * cx(o) + 9.0 * cu * cx(o) - 3.0 * gx);
      const double dy = wgt<double>(o) * rk * (3.0 * cy(o) + 9.0 * cu * cy(o) - 3.0 * gy);
      const double dz = wgt<double>(o) * rk * (3.0 * cz(o) + 9.0 * cu * cz(o) - 3.0 * gz);
      const double wk = flux ? A.w[-c - 2] : 0.0;
      const double coef = (A.nu[pidx((int32_t)p, o)] - wk) * (dx * K.n[0] + dy * K.n[1] + dz * K.n[2]) / rho;
#pragma unroll
      for (int j = 0; j < Q; ++j)
        m[j] += coef * (K.n[0] * (cx(j) - ux) + K.n[1] * (cy(j) - uy) + K.n[2] * (cz(j) - uz));
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) A.mu[pidx((int32_t)p, i)] = m[i];
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
  A.push = b.push;
  A.order = d.order;
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
  const unsigned grid = blocks_of(L.np);
  if (cfg.porous) {
    k_adj_collide<true><<<grid, kBlock, 0, s>>>(A);
    k_adj_stream<true><<<grid, kBlock, 0, s>>>(A);
  } else {
    k_adj_collide<false><<<grid, kBlock, 0, s>>>(A);
    k_adj_stream<false><<<grid, kBlock, 0, s>>>(A);
  }
  return hipGetLastError();
}

}  // namespace hlb
