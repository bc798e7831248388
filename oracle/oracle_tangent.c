/*
 * oracle_tangent.c -- tangent-linear (forward-mode) model of the FP64 CPU
 * oracle.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper defines no derivative.  This file differentiates the oracle's
 * forward update (oracle.c: moments eqs. (5)-(6), equilibrium eq. (4) with
 * the 1/2 factors, collision eq. (3a), push streaming eq. (3b) with the wall,
 * porous-wall, Ladd and ghost-density rules of Sec. 2.3) in forward mode: a
 * perturbation (df_0, dA, dphi) of the initial state, the per-step iolet
 * table values and the porosity is carried through every step next to the
 * state, and the objective's derivative in that direction is summed.
 *
 * It follows the forward update operation by operation (moments, then
 * equilibrium, then collision, then each link's rule), so it shares no
 * structure with the reference adjoint (oracle_adjoint.c), which transposes
 * explicit 19x19 Jacobians site by site.  The two meet in the dot-product
 * identity  dJ[v] = <grad J, v>,  which holds to rounding for any direction v
 * and pins the adjoint's transposition (indices, opposite directions, signs)
 * far more tightly than finite differences can.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int32_t TC[ORC_Q][3];
static double TW[ORC_Q];
static int32_t TOPP[ORC_Q];
static const double CS2 = 1.0 / 3.0;

/* c_i . v */
static double cdot(int i, const double *v) { return TC[i][0] * v[0] + TC[i][1] * v[1] + TC[i][2] * v[2]; }

/* Equilibrium eq. (4) at (rho, u) and its derivative in the direction
 * (drho, du):
 *   f^eq_i = w_i rho (1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2))
 *   d f^eq_i = w_i drho (...) + w_i rho (c.du/cs^2 + (c.u)(c.du)/cs^4 - u.du/cs^2) */
static void feq_tangent(double rho, const double *u, double drho, const double *du, double *feq, double *dfeq) {
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double udu = u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
  for (int i = 0; i < ORC_Q; ++i) {
    const double cu = cdot(i, u), cdu = cdot(i, du);
    const double shape = 1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
    feq[i] = TW[i] * rho * shape;
    dfeq[i] = TW[i] * drho * shape + TW[i] * rho * (cdu / CS2 + cu * cdu / (CS2 * CS2) - udu / CS2);
  }
}

/* Moments eqs. (5)-(6) and their derivative: rho = sum f, j = sum f c,
 * u = j / rho, du = (dj - drho u) / rho. */
static void moments_tangent(const double *f, const double *df, double *rho, double *u, double *drho, double *du) {
  double r = 0.0, dr = 0.0, j[3] = {0.0, 0.0, 0.0}, dj[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < ORC_Q; ++i) {
    r += f[i];
    dr += df[i];
    for (int a = 0; a < 3; ++a) {
      j[a] += f[i] * TC[i][a];
      dj[a] += df[i] * TC[i][a];
    }
  }
  *rho = r;
  *drho = dr;
  for (int a = 0; a < 3; ++a) {
    u[a] = j[a] / r;
    du[a] = (dj[a] - dr * u[a]) / r;
  }
}

/* Derivative of the wall shear stress of a site (definition of orc_macros)
 * in the direction df.  sigma = fac * Pi^neq, traction t = sigma n, s = t -
 * (t.n) n, WSS = |s|, so dWSS = s.ds / |s| (0 where s = 0). */
static double wss_tangent(const double *f, const double *df, const int32_t *nb, double tau) {
  double nv[3] = {0.0, 0.0, 0.0};
  int any = 0;
  for (int i = 1; i < ORC_Q; ++i)
    if (nb[i] == ORC_WALL) {
      any = 1;
      for (int a = 0; a < 3; ++a) nv[a] += TC[i][a];
    }
  const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  if (!any || nn == 0.0) return 0.0;
  for (int a = 0; a < 3; ++a) nv[a] /= nn;
  double rho, u[3], drho, du[3], feq[ORC_Q], dfeq[ORC_Q];
  moments_tangent(f, df, &rho, u, &drho, du);
  feq_tangent(rho, u, drho, du, feq, dfeq);
  double P[3][3] = {{0.0}}, dP[3][3] = {{0.0}};
  for (int i = 0; i < ORC_Q; ++i)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        P[a][b] += (f[i] - feq[i]) * TC[i][a] * TC[i][b];
        dP[a][b] += (df[i] - dfeq[i]) * TC[i][a] * TC[i][b];
      }
  const double fac = -(1.0 - 1.0 / (2.0 * tau));
  double t[3], dt[3];
  for (int a = 0; a < 3; ++a) {
    t[a] = fac * (P[a][0] * nv[0] + P[a][1] * nv[1] + P[a][2] * nv[2]);
    dt[a] = fac * (dP[a][0] * nv[0] + dP[a][1] * nv[1] + dP[a][2] * nv[2]);
  }
  const double tn = t[0] * nv[0] + t[1] * nv[1] + t[2] * nv[2];
  const double dtn = dt[0] * nv[0] + dt[1] * nv[1] + dt[2] * nv[2];
  double s[3], ds[3];
  for (int a = 0; a < 3; ++a) {
    s[a] = t[a] - tn * nv[a];
    ds[a] = dt[a] - dtn * nv[a];
  }
  const double w = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  if (w == 0.0) return 0.0;
  return (s[0] * ds[0] + s[1] * ds[1] + s[2] * ds[2]) / w;
}

/* One push update t -> t+1 with its tangent (serial: small cases only).
 * dA_t[k]: the perturbation of the table value iolet k uses at this step.
 * dQ (may be NULL) receives, per iolet, the derivative of the outflow of
 * this update, sum over the iolet's links of (d f'_i - d value returned). */
static int tl_step(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                   const orc_iolet *io, int32_t n_io, const double *phi, const double *dphi, int64_t t,
                   const double *dA_t, const double *f, const double *df, double *F, double *dF, double *dQ) {
  if (dQ)
    for (int k = 0; k < n_io; ++k) dQ[k] = 0.0;
  for (int64_t x = 0; x < n; ++x) {
    const double *fx = f + ORC_Q * x, *dfx = df + ORC_Q * x;
    double rho, u[3], drho, du[3], feq[ORC_Q], dfeq[ORC_Q], fp[ORC_Q], dfp[ORC_Q];
    moments_tangent(fx, dfx, &rho, u, &drho, du);
    feq_tangent(rho, u, drho, du, feq, dfeq);
    for (int i = 0; i < ORC_Q; ++i) {
      fp[i] = fx[i] - (fx[i] - feq[i]) / tau;
      dfp[i] = dfx[i] - (dfx[i] - dfeq[i]) / tau;
    }
    for (int i = 0; i < ORC_Q; ++i) {
      const int32_t y = nbr[ORC_Q * x + i];
      const int o = TOPP[i];
      if (y >= 0) {
        F[ORC_Q * (int64_t)y + i] = fp[i];
        dF[ORC_Q * (int64_t)y + i] = dfp[i];
        continue;
      }
      if (y == ORC_WALL) {
        /* (1 - phi) f'_i + phi w_i rho0 */
        const double ph = phi ? phi[x] : 0.0, dph = dphi ? dphi[x] : 0.0;
        F[ORC_Q * x + o] = (1.0 - ph) * fp[i] + ph * TW[i] * rho0;
        dF[ORC_Q * x + o] = (1.0 - ph) * dfp[i] - dph * fp[i] + dph * TW[i] * rho0;
        continue;
      }
      const int32_t k = -(y + 2);
      if (k < 0 || k >= n_io) return -1;
      const orc_iolet *K = io + k;
      const double a = orc_table_at(K, t), da = dA_t ? dA_t[k] : 0.0;
      double val, dval;
      if (K->kind == 0) {
        /* Ladd: f'_i - 2 w_i rho0 c_i.(a P(m)) / cs^2, m the link midpoint */
        const double m[3] = {coords[3 * x] + 0.5 * TC[i][0], coords[3 * x + 1] + 0.5 * TC[i][1],
                             coords[3 * x + 2] + 0.5 * TC[i][2]};
        double Pm[3];
        orc_iolet_profile(K, m, Pm);
        const double cP = cdot(i, Pm);
        val = fp[i] - 2.0 * TW[i] * rho0 * (a * cP) / CS2;
        dval = dfp[i] - 2.0 * TW[i] * rho0 * (da * cP) / CS2;
      } else {
        /* ghost density: f^eq_opp(i)(a, (u.n) n) */
        const double *nk = K->normal;
        const double un = u[0] * nk[0] + u[1] * nk[1] + u[2] * nk[2];
        const double dun = du[0] * nk[0] + du[1] * nk[1] + du[2] * nk[2];
        const double ug[3] = {un * nk[0], un * nk[1], un * nk[2]};
        const double dug[3] = {dun * nk[0], dun * nk[1], dun * nk[2]};
        double g[ORC_Q], dg[ORC_Q];
        feq_tangent(a, ug, da, dug, g, dg);
        val = g[o];
        dval = dg[o];
      }
      F[ORC_Q * x + o] = val;
      dF[ORC_Q * x + o] = dval;
      if (dQ) dQ[k] += dfp[i] - dval;
    }
  }
  return 0;
}

int orc_tl_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
               const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
               int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights, const double *f0,
               const double *df0, const double *dtab, const double *dphi, double *dJ) {
  if (objective != 0 && (objective != 1 || (n_io > 0 && !weights))) return -1;
  if (!f0 || !dJ || nsteps < 0) return -1;
  orc_lattice(&TC[0][0], TW, TOPP);
  const size_t sz = (size_t)ORC_Q * (size_t)n;
  double *a = (double *)malloc(sizeof(double) * sz), *b = (double *)malloc(sizeof(double) * sz);
  double *da = (double *)malloc(sizeof(double) * sz), *db = (double *)malloc(sizeof(double) * sz);
  double *dA_t = (double *)calloc(n_io > 0 ? (size_t)n_io : 1, sizeof(double));
  double *dQ = (double *)calloc(n_io > 0 ? (size_t)n_io : 1, sizeof(double));
  int rc = 0;
  double acc = 0.0;
  if (!a || !b || !da || !db || !dA_t || !dQ) {
    rc = -1;
    goto done;
  }
  memcpy(a, f0, sizeof(double) * sz);
  if (df0)
    memcpy(da, df0, sizeof(double) * sz);
  else
    memset(da, 0, sizeof(double) * sz);
  for (int64_t s = 0; s < nsteps; ++s) {
    const int64_t t = t0 + s;
    for (int k = 0; k < n_io; ++k) dA_t[k] = dtab ? dtab[(size_t)k * (size_t)nsteps + (size_t)s] : 0.0;
    const int in_window = t + 1 > obj_t0 && t + 1 <= obj_t1;
    if (tl_step(n, coords, nbr, tau, rho0, io, n_io, phi, dphi, t, dA_t, a, da, b, db,
                objective == 1 && in_window ? dQ : NULL) != 0) {
      rc = -1;
      goto done;
    }
    if (in_window) {
      if (objective == 1) {
        for (int k = 0; k < n_io; ++k) acc += weights[k] * dQ[k];
      } else {
        for (int64_t x = 0; x < n; ++x) acc += wss_tangent(b + ORC_Q * x, db + ORC_Q * x, nbr + ORC_Q * x, tau);
      }
    }
    double *tmp = a;
    a = b;
    b = tmp;
    tmp = da;
    da = db;
    db = tmp;
  }
  *dJ = acc;
done:
  free(a);
  free(b);
  free(da);
  free(db);
  free(dA_t);
  free(dQ);
  return rc;
}
