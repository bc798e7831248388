/*
 * oracle.c -- plain FP64 CPU reference of the sparse D3Q19 LBGK update.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Built with -ffp-contract=off so
 * that every multiply and add rounds separately, in source order.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D3Q19 (Sec. 2.2): i = 0 rest; 1-6 the axis directions; 7-18 the face
 * diagonals.  Opposite directions are adjacent. */
static const int32_t C[ORC_Q][3] = {
    {0, 0, 0},                                                        /* 0 */
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1}, {0, 0, -1}, /* 1-6 */
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},                /* 7-10 */
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},                /* 11-14 */
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};               /* 15-18 */
/* weights 1/3, 1/18, 1/36 (Sec. 2.2, after eq. (4)) */
static const double W[ORC_Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int32_t OPP[ORC_Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
static const double CS2 = 1.0 / 3.0; /* c_s = 1/sqrt(3) */

void orc_lattice(int32_t *c, double *w, int32_t *opp) {
  for (int i = 0; i < ORC_Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = C[i][a];
    w[i] = W[i];
    opp[i] = OPP[i];
  }
}

static double cdot(int i, const double *v) { return C[i][0] * v[0] + C[i][1] * v[1] + C[i][2] * v[2]; }

/* eq. (4): w_i rho (1 + (c.u)/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)) */
void orc_equilibrium(double rho, const double *u, double *feq) {
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < ORC_Q; ++i) {
    const double cu = cdot(i, u);
    feq[i] = W[i] * rho * (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* eqs. (5) and (6), summed in ascending i */
void orc_moments(const double *f, double *rho, double *u) {
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int i = 0; i < ORC_Q; ++i) {
    r += f[i];
    jx += f[i] * C[i][0];
    jy += f[i] * C[i][1];
    jz += f[i] * C[i][2];
  }
  *rho = r;
  u[0] = jx / r;
  u[1] = jy / r;
  u[2] = jz / r;
}

/* eq. (3a) with dt = 1: f' = f - (f - f^eq)/tau */
void orc_collide(const double *f, double tau, double *fout) {
  double rho, u[3], feq[ORC_Q];
  orc_moments(f, &rho, u);
  orc_equilibrium(rho, u, feq);
  for (int i = 0; i < ORC_Q; ++i) fout[i] = f[i] - (f[i] - feq[i]) / tau;
}

void orc_init(int64_t n, const double *rho, const double *u, double rho0, double *f) {
  for (int64_t x = 0; x < n; ++x) {
    const double zero[3] = {0.0, 0.0, 0.0};
    orc_equilibrium(rho ? rho[x] : rho0, u ? u + 3 * x : zero, f + ORC_Q * x);
  }
}

double orc_table_at(const orc_iolet *k, int64_t s) {
  if (k->table == NULL || k->table_len <= 0) return k->kind == 0 ? 0.0 : 1.0;
  return k->table[s % k->table_len];
}

/* Velocity profile of a Ladd iolet at point m per unit amplitude (Sec.
 * 2.3.2): a positional weight along the iolet's velocity direction.
 * Weight: parabolic in the distance d of m from the iolet axis,
 * max(0, 1 - d^2/R^2); uniform when R <= 0. */
void orc_iolet_profile(const orc_iolet *k, const double *m, double *P) {
  double wgt = 1.0;
  if (k->radius > 0.0) {
    const double r[3] = {m[0] - k->centre[0], m[1] - k->centre[1], m[2] - k->centre[2]};
    const double along = r[0] * k->normal[0] + r[1] * k->normal[1] + r[2] * k->normal[2];
    const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] - along * along;
    wgt = 1.0 - d2 / (k->radius * k->radius);
    if (wgt < 0.0) wgt = 0.0;
  }
  const double *v = k->vdir;
  if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0) v = k->normal;
  P[0] = wgt * v[0];
  P[1] = wgt * v[1];
  P[2] = wgt * v[2];
}

/* Velocity imposed at m and step s: the amplitude A_k(s) times the profile. */
static void iolet_velocity(const orc_iolet *k, const double *m, int64_t s, double *U) {
  double P[3];
  orc_iolet_profile(k, m, P);
  const double a = orc_table_at(k, s);
  U[0] = a * P[0];
  U[1] = a * P[1];
  U[2] = a * P[2];
}

/* Compensated (Kahan) accumulator. */
typedef struct { double s, c; } kahan;
static void kadd(kahan *k, double v) {
  const double y = v - k->c;
  const double t = k->s + y;
  k->c = (t - k->s) - y;
  k->s = t;
}

/* The population an iolet returns to site x (coordinates xc) in direction
 * opp(i) when the post-collision f'_i(x) = fp[i] leaves through it during the
 * update t -> t+1; u is the site's velocity at t.
 *   Ladd (Sec. 2.3.2): bounce-back plus -2 w_i rho c_i.U / cs^2, rho = rho0
 *     (or, with rho_local, the site's density rho_x at t), U taken at the
 *     link midpoint x + c_i/2;
 *   ghost density (Sec. 2.3.2): the equilibrium at the iolet density
 *     rho_k(t) and the site velocity projected on the iolet normal. */
static double iolet_fill(const orc_iolet *K, const int32_t *xc, int i, int64_t t, double rho0, double rho_x,
                         const double *fp, const double *u) {
  if (K->kind == 0) {
    const double m[3] = {xc[0] + 0.5 * C[i][0], xc[1] + 0.5 * C[i][1], xc[2] + 0.5 * C[i][2]};
    double U[3];
    iolet_velocity(K, m, t, U);
    const double rw = K->rho_local ? rho_x : rho0;
    return fp[i] - 2.0 * W[i] * rw * cdot(i, U) / CS2;
  }
  const double *nk = K->normal;
  const double un = u[0] * nk[0] + u[1] * nk[1] + u[2] * nk[2];
  const double ug[3] = {un * nk[0], un * nk[1], un * nk[2]};
  double fg[ORC_Q];
  orc_equilibrium(orc_table_at(K, t), ug, fg);
  return fg[OPP[i]];
}

int orc_iolet_flux(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                   const orc_iolet *io, int32_t n_io, int64_t t, const double *f, double *Q) {
  for (int k = 0; k < n_io; ++k) Q[k] = 0.0;
  int bad = 0;
  /* serial over sites: a fixed summation order, small cases only */
  for (int64_t x = 0; x < n; ++x) {
    const double *fx = f + ORC_Q * x;
    double rho, u[3], fp[ORC_Q];
    int any = 0;
    for (int i = 0; i < ORC_Q; ++i) any |= nbr[ORC_Q * x + i] < ORC_WALL;
    if (!any) continue;
    orc_moments(fx, &rho, u);
    orc_collide(fx, tau, fp);
    for (int i = 0; i < ORC_Q; ++i) {
      const int32_t y = nbr[ORC_Q * x + i];
      if (y >= ORC_WALL) continue;
      const int32_t k = -(y + 2);
      if (k < 0 || k >= n_io) { bad = 1; continue; }
      Q[k] += fp[i] - iolet_fill(io + k, coords + 3 * x, i, t, rho0, rho, fp, u);
    }
  }
  return bad ? -1 : 0;
}

int orc_step(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
             const orc_iolet *io, int32_t n_io, const double *phi, int64_t t, const double *f,
             double *F, double *flux_out, int32_t *write_count) {
  int bad = 0;
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  kahan *part = (kahan *)calloc((size_t)nthreads, sizeof(kahan));
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    kahan acc = {0.0, 0.0};
#pragma omp for schedule(static)
    for (int64_t x = 0; x < n; ++x) {
      const double *fx = f + ORC_Q * x;
      double rho, u[3], feq[ORC_Q], fp[ORC_Q];
      /* collision (eq. 3a) from the moments of f(x, t) */
      orc_moments(fx, &rho, u);
      orc_equilibrium(rho, u, feq);
      for (int i = 0; i < ORC_Q; ++i) fp[i] = fx[i] - (fx[i] - feq[i]) / tau;
      /* streaming (eq. 3b) with the boundary rules applied in the same pass */
      for (int i = 0; i < ORC_Q; ++i) {
        const int32_t y = nbr[ORC_Q * x + i];
        int64_t slot;
        double val;
        if (y >= 0) {
          slot = ORC_Q * (int64_t)y + i;
          val = fp[i];
        } else if (y == ORC_WALL) {
          /* mid-link bounce-back (Sec. 2.3.1): the population returns to x
           * reversed.  A porous wall site (porosity phi) lets a fraction phi
           * leak to a reservoir at rest density rho0 instead. */
          const double ph = phi ? phi[x] : 0.0;
          slot = ORC_Q * x + OPP[i];
          val = (1.0 - ph) * fp[i] + ph * W[i] * rho0;
          kadd(&acc, val - fp[i]);
        } else {
          const int32_t k = -(y + 2);
          if (k < 0 || k >= n_io) { bad = 1; continue; }
          slot = ORC_Q * x + OPP[i];
          val = iolet_fill(io + k, coords + 3 * x, i, t, rho0, rho, fp, u);
          kadd(&acc, val - fp[i]);
        }
        F[slot] = val;
        if (write_count) {
#pragma omp atomic
          write_count[slot] += 1;
        }
      }
    }
    part[tid] = acc;
  }
  if (flux_out) {
    kahan tot = {0.0, 0.0};
    for (int i = 0; i < nthreads; ++i) {
      kadd(&tot, part[i].s);
      kadd(&tot, -part[i].c);
    }
    *flux_out = tot.s;
  }
  free(part);
  return bad ? -1 : 0;
}

int orc_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
            const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
            double *f, double *work, double *flux_sum) {
  double *a = f, *b = work;
  kahan acc = {flux_sum ? *flux_sum : 0.0, 0.0};
  for (int64_t s = 0; s < nsteps; ++s) {
    double fl = 0.0;
    if (orc_step(n, coords, nbr, tau, rho0, io, n_io, phi, t0 + s, a, b, &fl, NULL) != 0) return -1;
    kadd(&acc, fl);
    double *tmp = a;
    a = b;
    b = tmp;
  }
  if (a != f) memcpy(f, a, sizeof(double) * ORC_Q * (size_t)n);
  if (flux_sum) *flux_sum = acc.s;
  return 0;
}

/* Wall shear stress at a site with wall links (not defined by the paper):
 * deviatoric stress from the non-equilibrium second moment,
 *   sigma = -(1 - 1/(2 tau)) sum_i (f_i - f_i^eq) c_i c_i,
 * wall normal n = normalised sum of the wall-link directions, traction
 * t = sigma n, WSS = |t - (t.n) n|. */
static double site_wss(const double *fx, const int32_t *nb, double tau) {
  double nv[3] = {0.0, 0.0, 0.0};
  int any = 0;
  for (int i = 1; i < ORC_Q; ++i)
    if (nb[i] == ORC_WALL) {
      any = 1;
      nv[0] += C[i][0];
      nv[1] += C[i][1];
      nv[2] += C[i][2];
    }
  if (!any) return 0.0;
  const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  if (nn == 0.0) return 0.0;
  nv[0] /= nn;
  nv[1] /= nn;
  nv[2] /= nn;
  double rho, u[3], feq[ORC_Q];
  orc_moments(fx, &rho, u);
  orc_equilibrium(rho, u, feq);
  double P[3][3] = {{0.0}};
  for (int i = 0; i < ORC_Q; ++i) {
    const double d = fx[i] - feq[i];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) P[a][b] += d * C[i][a] * C[i][b];
  }
  const double fac = -(1.0 - 1.0 / (2.0 * tau));
  double tr[3];
  for (int a = 0; a < 3; ++a) tr[a] = fac * (P[a][0] * nv[0] + P[a][1] * nv[1] + P[a][2] * nv[2]);
  const double tn = tr[0] * nv[0] + tr[1] * nv[1] + tr[2] * nv[2];
  const double s0 = tr[0] - tn * nv[0], s1 = tr[1] - tn * nv[1], s2 = tr[2] - tn * nv[2];
  return sqrt(s0 * s0 + s1 * s1 + s2 * s2);
}

void orc_macros(int64_t n, const int32_t *nbr, double tau, const double *f, double *rho, double *u,
                double *wss) {
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < n; ++x) {
    double r, v[3];
    orc_moments(f + ORC_Q * x, &r, v);
    if (rho) rho[x] = r;
    if (u) {
      u[3 * x] = v[0];
      u[3 * x + 1] = v[1];
      u[3 * x + 2] = v[2];
    }
    if (wss) wss[x] = site_wss(f + ORC_Q * x, nbr + ORC_Q * x, tau);
  }
}

double orc_mass(int64_t n, const double *f) {
  kahan acc = {0.0, 0.0};
  for (int64_t k = 0; k < ORC_Q * n; ++k) kadd(&acc, f[k]);
  return acc.s;
}

int32_t orc_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

double orc_wss_sum(int64_t n, const int32_t *nbr, double tau, const double *f) {
  kahan acc = {0.0, 0.0};
  for (int64_t x = 0; x < n; ++x) kadd(&acc, site_wss(f + ORC_Q * x, nbr + ORC_Q * x, tau));
  return acc.s;
}
