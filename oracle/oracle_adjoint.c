/*
 * oracle_adjoint.c -- reference adjoint of the FP64 CPU oracle.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper defines no adjoint.  This file differentiates the oracle's own
 * update (push order, pre-collision state, oracle.c) by hand:
 *   f_{t+1} = S_t(f_t; A(t), phi)
 * where S_t is the collision of every site (eq. (3a), equilibrium eq. (4))
 * followed by the scatter of eq. (3b) with the boundary rules of Sec. 2.3.
 * With mu_t = dJ/df_t (J as in oracle.h),
 *   mu_t = (dS_t/df_t)^T mu_{t+1} + dJ_t/df_t,
 *   dJ/dA_k(t) = (dS_t/dA_k)^T mu_{t+1} + dJ_t/dA_k(t),
 *   dJ/dphi_x += (dS_t/dphi_x)^T mu_{t+1},
 * A_k(t) the table value of iolet k (amplitude or ghost density).  The WSS
 * objective depends on f_t only; the outflow objective of the update
 * t -> t+1 depends on f_t and A_k(t) directly.
 * All forward states are kept in memory (no checkpointing): small cases only.
 * The Jacobians are written out as explicit 19x19 matrices.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

static int32_t LC[ORC_Q][3];
static double LW[ORC_Q];
static int32_t LOPP[ORC_Q];
static const double CS2 = 1.0 / 3.0;

static void lattice_init(void) { orc_lattice(&LC[0][0], LW, LOPP); }

/* D[i][j] = d f^eq_i / d f_j at the state f (rho, u its moments):
 * f^eq_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u), rho = sum f,
 * u = (sum f c)/rho, so d rho/d f_j = 1 and d u/d f_j = (c_j - u)/rho. */
static void dfeq_df(const double *f, double D[ORC_Q][ORC_Q]) {
  double rho, u[3], feq[ORC_Q];
  orc_moments(f, &rho, u);
  orc_equilibrium(rho, u, feq);
  for (int i = 0; i < ORC_Q; ++i) {
    const double cu = LC[i][0] * u[0] + LC[i][1] * u[1] + LC[i][2] * u[2];
    double g[3]; /* d f^eq_i / d u */
    for (int a = 0; a < 3; ++a) g[a] = LW[i] * rho * (3.0 * LC[i][a] + 9.0 * cu * LC[i][a] - 3.0 * u[a]);
    for (int j = 0; j < ORC_Q; ++j) {
      double du = 0.0;
      for (int a = 0; a < 3; ++a) du += g[a] * (LC[j][a] - u[a]) / rho;
      D[i][j] = feq[i] / rho + du;
    }
  }
}

/* Wall shear stress of site state f (definition of orc_macros) and its
 * gradient with respect to f; grad = 0 where the tangential traction is 0. */
static double wss_and_grad(const double *f, const int32_t *nb, double tau, double *grad) {
  for (int j = 0; j < ORC_Q; ++j) grad[j] = 0.0;
  double nv[3] = {0.0, 0.0, 0.0};
  int any = 0;
  for (int i = 1; i < ORC_Q; ++i)
    if (nb[i] == ORC_WALL) {
      any = 1;
      for (int a = 0; a < 3; ++a) nv[a] += LC[i][a];
    }
  const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  if (!any || nn == 0.0) return 0.0;
  for (int a = 0; a < 3; ++a) nv[a] /= nn;
  double rho, u[3], feq[ORC_Q];
  orc_moments(f, &rho, u);
  orc_equilibrium(rho, u, feq);
  double P[3][3] = {{0.0}};
  for (int i = 0; i < ORC_Q; ++i)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) P[a][b] += (f[i] - feq[i]) * LC[i][a] * LC[i][b];
  const double fac = -(1.0 - 1.0 / (2.0 * tau));
  double t[3];
  for (int a = 0; a < 3; ++a) t[a] = fac * (P[a][0] * nv[0] + P[a][1] * nv[1] + P[a][2] * nv[2]);
  const double tn = t[0] * nv[0] + t[1] * nv[1] + t[2] * nv[2];
  double s[3];
  for (int a = 0; a < 3; ++a) s[a] = t[a] - tn * nv[a];
  const double w = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  if (w == 0.0) return 0.0;
  /* d WSS / d (f_i - feq_i) = fac (c_i.n)(e.c_i), e = s / |s| */
  double wd[ORC_Q];
  for (int i = 0; i < ORC_Q; ++i) {
    const double cn = LC[i][0] * nv[0] + LC[i][1] * nv[1] + LC[i][2] * nv[2];
    const double ce = (LC[i][0] * s[0] + LC[i][1] * s[1] + LC[i][2] * s[2]) / w;
    wd[i] = fac * cn * ce;
  }
  double D[ORC_Q][ORC_Q];
  dfeq_df(f, D);
  for (int j = 0; j < ORC_Q; ++j) {
    double v = wd[j];
    for (int i = 0; i < ORC_Q; ++i) v -= wd[i] * D[i][j];
    grad[j] = v;
  }
  return w;
}

/* Transpose of one push update t -> t+1 (oracle.c, orc_step), site by site:
 * mu_out[x] = (dS/df_t(x))^T mu_next; Ladd and porosity parameter
 * derivatives are added to dA_part (per thread, [n_io]) and dJ_dphi. */
static int adj_step(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                    const orc_iolet *io, int32_t n_io, const double *phi, int64_t t, const double *f,
                    const double *mu_next, const double *wflux, double *mu_out, double *dA, double *dJ_dphi) {
  int bad = 0;
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  double *part = (double *)calloc((size_t)nthreads * (n_io > 0 ? n_io : 1), sizeof(double));
  if (!part) return -1;
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double *myA = part + (size_t)tid * (n_io > 0 ? n_io : 1);
#pragma omp for schedule(static)
    for (int64_t x = 0; x < n; ++x) {
      const double *fx = f + ORC_Q * x;
      double rho, u[3], feq[ORC_Q], fp[ORC_Q];
      orc_moments(fx, &rho, u);
      orc_equilibrium(rho, u, feq);
      for (int i = 0; i < ORC_Q; ++i) fp[i] = fx[i] - (fx[i] - feq[i]) / tau;
      double a[ORC_Q];   /* dJ / d f'_i(x) */
      double dpre[ORC_Q]; /* dJ / d f_j(x) through the pressure rule's u(x) */
      for (int i = 0; i < ORC_Q; ++i) a[i] = dpre[i] = 0.0;
      for (int i = 0; i < ORC_Q; ++i) {
        const int32_t y = nbr[ORC_Q * x + i];
        if (y >= 0) {
          a[i] = mu_next[ORC_Q * (int64_t)y + i];
        } else if (y == ORC_WALL) {
          const double m = mu_next[ORC_Q * x + LOPP[i]];
          const double ph = phi ? phi[x] : 0.0;
          a[i] = (1.0 - ph) * m;
          if (dJ_dphi) dJ_dphi[x] += m * (LW[i] * rho0 - fp[i]);
        } else {
          const int32_t k = -(y + 2);
          if (k < 0 || k >= n_io) { bad = 1; continue; }
          const orc_iolet *K = io + k;
          const double m = mu_next[ORC_Q * x + LOPP[i]];
          /* outflow objective: this link adds f'_i - value to Q_k */
          const double wk = wflux ? wflux[k] : 0.0;
          if (K->kind == 0) {
            /* value = f'_i + A_k(t) * (-2 w_i rho0 c_i.P / cs^2): the outflow
             * does not depend on f'_i */
            a[i] = m;
            const double mp[3] = {coords[3 * x] + 0.5 * LC[i][0], coords[3 * x + 1] + 0.5 * LC[i][1],
                                  coords[3 * x + 2] + 0.5 * LC[i][2]};
            double P[3];
            orc_iolet_profile(K, mp, P);
            const double cP = LC[i][0] * P[0] + LC[i][1] * P[1] + LC[i][2] * P[2];
            myA[k] += (m - wk) * (-2.0 * LW[i] * rho0 * cP / CS2);
          } else {
            /* value = f^eq_o(rho_k, ug), o = opp(i), ug = (u.n) n */
            a[i] = wk;
            const int o = LOPP[i];
            const double *nk = K->normal;
            const double un = u[0] * nk[0] + u[1] * nk[1] + u[2] * nk[2];
            const double ug[3] = {un * nk[0], un * nk[1], un * nk[2]};
            const double rk = orc_table_at(K, t);
            double f1[ORC_Q]; /* d value / d rho_k = f^eq_o(1, ug) */
            orc_equilibrium(1.0, ug, f1);
            myA[k] += (m - wk) * f1[o];
            const double cu = LC[o][0] * ug[0] + LC[o][1] * ug[1] + LC[o][2] * ug[2];
            double g[3]; /* d f^eq_o / d ug */
            for (int b = 0; b < 3; ++b) g[b] = LW[o] * rk * (3.0 * LC[o][b] + 9.0 * cu * LC[o][b] - 3.0 * ug[b]);
            const double gn = g[0] * nk[0] + g[1] * nk[1] + g[2] * nk[2];
            /* d ug / d f_j = n (n . (c_j - u)) / rho */
            for (int j = 0; j < ORC_Q; ++j) {
              const double ncj = nk[0] * (LC[j][0] - u[0]) + nk[1] * (LC[j][1] - u[1]) + nk[2] * (LC[j][2] - u[2]);
              dpre[j] += (m - wk) * gn * ncj / rho;
            }
          }
        }
      }
      /* collision Jacobian: d f'_i / d f_j = (1 - 1/tau) delta_ij + (1/tau) d feq_i / d f_j */
      double D[ORC_Q][ORC_Q];
      dfeq_df(fx, D);
      for (int j = 0; j < ORC_Q; ++j) {
        double v = (1.0 - 1.0 / tau) * a[j];
        for (int i = 0; i < ORC_Q; ++i) v += a[i] * D[i][j] / tau;
        mu_out[ORC_Q * x + j] = v + dpre[j];
      }
    }
  }
  for (int th = 0; th < nthreads; ++th)
    for (int k = 0; k < n_io; ++k) dA[k] += part[(size_t)th * n_io + k];
  free(part);
  return bad ? -1 : 0;
}

/* Windkessel outlets (an extension; the forward model is the oracle's
 * Python driver, Problem.run_windkessel): pressure iolet k with wk_on[k] set
 * takes at step s the density rho_k(s) of its state, and after the update
 * s -> s+1 with outflow Q_k(s) (orc_iolet_flux at s)
 *   X(s+1)     = X(s) + (Q - X/R2)/C   (C > 0; no X/R2 term if R2 = 0),
 *                R2 Q                   (C = 0),
 *   rho_k(s+1) = rho_ref + R1 Q + X(s+1),
 * from X(0) = X0, rho_k(0) = rho_ref + X0; wk[k] = (rho_ref, R1, C, R2, X0).
 * Its adjoint is a scalar recurrence per outlet, backwards in s:
 *   LX(s+1) = Lr(s+1) + kappa LX(s+2),  kappa = dX(s+2)/dX(s+1)
 *             (1 - 1/(R2 C), 1 if R2 = 0, 0 if C = 0),
 *   dJ/dQ_k(s) = R1 Lr(s+1) + dX(s+1)/dQ LX(s+1)   (1/C, or R2 if C = 0),
 * Lr(s) the derivative with respect to the density used at step s (the
 * table-value derivative of that step, which already carries the outflow
 * weights of step s), Lr(N) = LX(N) = LX(N+1) = 0.  dJ/dQ_k(s) enters the
 * adjoint step of the update s -> s+1 as an outflow weight, added to the
 * objective's own weight. */
static int adj_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                   const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
                   int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights,
                   const int32_t *wk_on, const double *wk, const double *f0, double *J, double *dJ_dA,
                   double *dJ_dphi, double *dJ_df0) {
  if (objective != 0 && (objective != 1 || (n_io > 0 && !weights))) return -1;
  int any_wk = 0;
  for (int k = 0; wk_on && k < n_io; ++k) {
    if (!wk_on[k]) continue;
    if (io[k].kind != 1 || !wk || wk[5 * k + 2] < 0.0) return -1;
    any_wk = 1;
  }
  const int wss = objective == 0;
  lattice_init();
  const size_t sz = (size_t)ORC_Q * (size_t)n;
  const size_t nk = n_io > 0 ? (size_t)n_io : 1;
  double *F = (double *)malloc(sizeof(double) * sz * (size_t)(nsteps + 1));
  double *mu = (double *)calloc(sz, sizeof(double));
  double *mu2 = (double *)calloc(sz, sizeof(double));
  double *gr = (double *)malloc(sizeof(double) * sz);
  double *dA = (double *)calloc(nk, sizeof(double));
  double *Qk = (double *)calloc(nk, sizeof(double));
  double *weff = (double *)calloc(nk, sizeof(double));
  double *Lr = (double *)calloc(nk, sizeof(double));  /* Lr(s+1) */
  double *LX = (double *)calloc(nk, sizeof(double));  /* LX(s+2), then LX(s+1) */
  double *rh = (double *)calloc(nk * (size_t)(nsteps + 1), sizeof(double)); /* rho_k(s) */
  orc_iolet *iw = (orc_iolet *)malloc(sizeof(orc_iolet) * nk);
  int rc = -1;
  if (!F || !mu || !mu2 || !gr || !dA || !Qk || !weff || !Lr || !LX || !rh || !iw) goto done;
  if (n_io > 0) memcpy(iw, io, sizeof(orc_iolet) * (size_t)n_io);
#define WK_AT(s)                                                             \
  for (int k = 0; any_wk && k < n_io; ++k)                                   \
    if (wk_on[k]) {                                                          \
      iw[k].table = rh + (size_t)k * (size_t)(nsteps + 1) + (size_t)(s);    \
      iw[k].table_len = 1;                                                   \
    }
  /* forward, storing every state (and the outlets' densities) */
  {
    double *X = Lr; /* the outlets' X during the forward sweep (reset below) */
    for (int k = 0; any_wk && k < n_io; ++k)
      if (wk_on[k]) {
        X[k] = wk[5 * k + 4];
        rh[(size_t)k * (size_t)(nsteps + 1)] = wk[5 * k] + wk[5 * k + 4];
      }
    memcpy(F, f0, sizeof(double) * sz);
    for (int64_t s = 0; s < nsteps; ++s) {
      WK_AT(s);
      if (any_wk && orc_iolet_flux(n, coords, nbr, tau, rho0, iw, n_io, t0 + s, F + sz * s, Qk) != 0) goto done;
      if (orc_step(n, coords, nbr, tau, rho0, iw, n_io, phi, t0 + s, F + sz * s, F + sz * (s + 1), NULL, NULL) != 0)
        goto done;
      for (int k = 0; any_wk && k < n_io; ++k) {
        if (!wk_on[k]) continue;
        const double *P = wk + 5 * k;
        X[k] = P[2] > 0.0 ? X[k] + (Qk[k] - (P[3] > 0.0 ? X[k] / P[3] : 0.0)) / P[2] : P[3] * Qk[k];
        rh[(size_t)k * (size_t)(nsteps + 1) + (size_t)(s + 1)] = P[0] + P[1] * Qk[k] + X[k];
      }
    }
    for (size_t k = 0; k < nk; ++k) Lr[k] = 0.0;
  }
  /* objective: WSS of the state at t, or the weighted outflow of the update
   * t-1 -> t, for each t in the window */
  {
    double Jsum = 0.0, Jc = 0.0;
    for (int64_t s = 1; s <= nsteps; ++s) {
      const int64_t t = t0 + s;
      if (t <= obj_t0 || t > obj_t1) continue;
      double v = 0.0;
      if (wss) {
        v = orc_wss_sum(n, nbr, tau, F + sz * s);
      } else {
        WK_AT(s - 1);
        if (orc_iolet_flux(n, coords, nbr, tau, rho0, iw, n_io, t - 1, F + sz * (s - 1), Qk) != 0) goto done;
        for (int k = 0; k < n_io; ++k) v += weights[k] * Qk[k];
      }
      const double y = v - Jc, tt = Jsum + y;
      Jc = (tt - Jsum) - y;
      Jsum = tt;
    }
    *J = Jsum;
  }
  if (dJ_dphi) memset(dJ_dphi, 0, sizeof(double) * (size_t)n);
  if (dJ_dA) memset(dJ_dA, 0, sizeof(double) * (size_t)(n_io > 0 ? n_io : 0) * (size_t)nsteps);
  /* mu = dJ/df_T */
  if (wss && t0 + nsteps > obj_t0 && t0 + nsteps <= obj_t1) {
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < n; ++x) wss_and_grad(F + sz * nsteps + ORC_Q * x, nbr + ORC_Q * x, tau, mu + ORC_Q * x);
  }
  for (int64_t s = nsteps - 1; s >= 0; --s) {
    for (int k = 0; k < n_io; ++k) dA[k] = 0.0;
    /* the outflow of the update t0+s -> t0+s+1 counts if t0+s+1 is in the window */
    const int flux_here = !wss && t0 + s + 1 > obj_t0 && t0 + s + 1 <= obj_t1;
    for (int k = 0; k < n_io; ++k) weff[k] = flux_here ? weights[k] : 0.0;
    for (int k = 0; any_wk && k < n_io; ++k) {
      if (!wk_on[k]) continue;
      const double *P = wk + 5 * k;
      const double kappa = P[2] > 0.0 ? 1.0 - (P[3] > 0.0 ? 1.0 / (P[3] * P[2]) : 0.0) : 0.0;
      LX[k] = Lr[k] + kappa * LX[k];
      weff[k] += P[1] * Lr[k] + (P[2] > 0.0 ? 1.0 / P[2] : P[3]) * LX[k];
    }
    WK_AT(s);
    if (adj_step(n, coords, nbr, tau, rho0, iw, n_io, phi, t0 + s, F + sz * s, mu,
                 (flux_here || any_wk) ? weff : NULL, mu2, dA, dJ_dphi) != 0)
      goto done;
    for (int k = 0; k < n_io; ++k) Lr[k] = dA[k];
    if (dJ_dA)
      for (int k = 0; k < n_io; ++k) dJ_dA[(size_t)k * nsteps + s] = dA[k];
    const int64_t t = t0 + s;
    if (wss && s >= 1 && t > obj_t0 && t <= obj_t1) {
#pragma omp parallel for schedule(static)
      for (int64_t x = 0; x < n; ++x) {
        wss_and_grad(F + sz * s + ORC_Q * x, nbr + ORC_Q * x, tau, gr + ORC_Q * x);
        for (int j = 0; j < ORC_Q; ++j) mu2[ORC_Q * x + j] += gr[ORC_Q * x + j];
      }
    }
    double *tmp = mu;
    mu = mu2;
    mu2 = tmp;
  }
#undef WK_AT
  if (dJ_df0) memcpy(dJ_df0, mu, sizeof(double) * sz);
  rc = 0;
done:
  free(F); free(mu); free(mu2); free(gr); free(dA); free(Qk); free(weff); free(Lr); free(LX); free(rh); free(iw);
  return rc;
}

int orc_adj_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
                int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights, const double *f0,
                double *J, double *dJ_dA, double *dJ_dphi, double *dJ_df0) {
  return adj_run(n, coords, nbr, tau, rho0, io, n_io, phi, t0, nsteps, obj_t0, obj_t1, objective, weights, NULL,
                 NULL, f0, J, dJ_dA, dJ_dphi, dJ_df0);
}

int orc_adj_run_wk(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                   const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
                   int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights, const int32_t *wk_on,
                   const double *wk, const double *f0, double *J, double *dJ_dA, double *dJ_dphi, double *dJ_df0) {
  return adj_run(n, coords, nbr, tau, rho0, io, n_io, phi, t0, nsteps, obj_t0, obj_t1, objective, weights, wk_on, wk,
                 f0, J, dJ_dA, dJ_dphi, dJ_df0);
}
