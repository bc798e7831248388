/*
 * oracle.h -- plain FP64 CPU reference of the sparse D3Q19 LBGK update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code; only the test suite, the smoke check and the CPU legs
 * of the benchmark (baseline, timing table) use it.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * What it computes (Zacharoudiou, McCullough, Coveney, "Development and
 * performance of a HemeLB GPU code for human-scale blood flow simulation"):
 *   - D3Q19 lattice, weights 1/3, 1/18, 1/36, c_s^2 = 1/3       (Sec. 2.2)
 *   - BGK collision, eq. (3a); streaming, eq. (3b)               (Sec. 2.2)
 *   - equilibrium, eq. (4), read with the usual 1/2 factors on the
 *     second-order terms (the printed form lacks them; see the readings)
 *   - density and momentum moments, eqs. (5), (6)
 *   - mid-link bounce-back at walls                              (Sec. 2.3.1)
 *   - Ladd velocity iolets and ghost-density pressure iolets     (Sec. 2.3.2)
 *   - push order: collide, then scatter, with the boundary rules applied in
 *     the same pass                                               (Sec. 3.1)
 * Layout: array of structures f[x*19 + i], sites in input order.
 *
 * Extensions the paper does not define, each stated where it is used:
 * wall shear stress, per-wall-site porosity, the mass-balance bookkeeping,
 * and the adjoint and tangent-linear models of oracle_adjoint.c and
 * oracle_tangent.c.
 *
 * Pins: see tests/test_oracle_*.py.  The pressure-iolet ghost velocity
 * (site velocity projected on the iolet normal) and the wall normal used by
 * the shear stress are readings with no physical pin: parity unpinned for
 * those two choices beyond both codes implementing the written definition.
 * The velocity-iolet density (reference density rho0, or the site's own
 * density with rho_local set) is pinned by a Couette column away from rho0.
 */
#ifndef HLB_ORACLE_H
#define HLB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_Q 19
#define ORC_WALL (-1) /* link code of a wall; iolet k is -(2+k) */

typedef struct {
  int32_t kind;      /* 0: velocity (Ladd), 1: pressure (ghost density) */
  int32_t role;      /* 0: inlet, 1: outlet (classification only) */
  double centre[3];  /* point on the iolet plane */
  double normal[3];  /* unit normal pointing into the fluid */
  double radius;     /* > 0: parabolic weight max(0, 1 - d^2/R^2); <= 0: weight 1 */
  double vdir[3];    /* direction of the imposed velocity; all zero: normal */
  const double *table; /* per-step amplitude A_k(s) or ghost density rho_k(s) */
  int64_t table_len;   /* value at step s is table[s mod table_len] */
  int32_t rho_local;   /* velocity kind: 1 = the Ladd term takes the site's own
                          density at t, 0 = the reference density rho0 (the
                          forward update only; the adjoint and tangent codes
                          take rho0) */
} orc_iolet;

/* Lattice constants as the oracle uses them (for the tests). */
void orc_lattice(int32_t *c /*[19][3]*/, double *w /*[19]*/, int32_t *opp /*[19]*/);

/* eq. (4) with the 1/2 factors. */
void orc_equilibrium(double rho, const double *u, double *feq);
/* eqs. (5), (6): rho = sum f, rho u = sum f c. */
void orc_moments(const double *f, double *rho, double *u);
/* eq. (3a) with dt = 1. */
void orc_collide(const double *f, double tau, double *fout);

/* f(x,0) = f^eq(rho(x), u(x)); rho, u may be NULL (rho0, 0).  Sec. 3.1 step 1. */
void orc_init(int64_t n, const double *rho, const double *u, double rho0, double *f);

/* One update t -> t+1 (push).  f: pre-collision state at t, F: state at t+1.
 * phi: per-site porosity (read at wall links) or NULL.  flux_out: receives
 * the mass the boundary rules added this step, sum over boundary links of
 * (value filled in - post-collision value that left).  write_count: NULL, or
 * an int32 array [n*19] that is incremented once per write of a slot.
 * Returns 0, or -1 on a bad link code. */
int orc_step(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
             const orc_iolet *io, int32_t n_io, const double *phi, int64_t t, const double *f,
             double *F, double *flux_out, int32_t *write_count);

/* Net outflow through each iolet during the update t -> t+1 from the
 * pre-collision state f at t (not a rule of the paper; the outlet-flux
 * objective): Q[k] = sum over the links of iolet k of (post-collision
 * population that leaves - population the iolet returns).  Summed over all
 * iolets it is the mass the step loses (no porosity).  Returns 0, or -1 on
 * a bad link code. */
int orc_iolet_flux(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                   const orc_iolet *io, int32_t n_io, int64_t t, const double *f, double *Q);

/* nsteps updates starting at time t0; f holds the state at t0 on entry and at
 * t0+nsteps on return (work: scratch of n*19 doubles).  *flux_sum (may be
 * NULL) is increased by the boundary mass flux of every step. */
int orc_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
            const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
            double *f, double *work, double *flux_sum);

/* Density, velocity and wall shear stress of state f (pre-collision).
 * wss is 0 at sites without a wall link.  Any output may be NULL. */
void orc_macros(int64_t n, const int32_t *nbr, double tau, const double *f, double *rho, double *u,
                double *wss);

/* Total mass sum_x sum_i f_i (compensated summation). */
double orc_mass(int64_t n, const double *f);

/* Table value of iolet k at step s (table[s mod len]). */
double orc_table_at(const orc_iolet *k, int64_t s);
/* Ladd velocity profile per unit amplitude at point m: weight times direction. */
void orc_iolet_profile(const orc_iolet *k, const double *m, double *P);

/* Reference adjoint (oracle_adjoint.c).  Objective, for t in (obj_t0,
 * obj_t1] with t0 < t <= t0 + nsteps:
 *   objective 0: J = sum over t of the sum of WSS(x, t) over the sites with
 *                wall links (WSS of the pre-collision state at t as in
 *                orc_macros);
 *   objective 1: J = sum over t of sum_k weights[k] Q_k, Q_k the outflow of
 *                iolet k during the update t-1 -> t (orc_iolet_flux).
 * From the state f0 at t0, run nsteps forward (storing every state), then
 * the adjoint sweep.  Outputs: *J; dJ_dtab [n_io][nsteps]: derivative with
 * respect to the table value iolet k uses at step t0+s (the amplitude A_k of
 * a velocity iolet, the ghost density rho_k of a pressure iolet); dJ_dphi
 * [n]: derivative with respect to each site's porosity (zero at sites without
 * wall links); dJ_df0 [n*19] (may be NULL): derivative with respect to the
 * initial state f0.  phi may be NULL (no porosity, derivative still at
 * phi = 0).  Returns 0, or -1 on a bad argument, link code or allocation
 * failure. */
int orc_adj_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
                int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights, const double *f0,
                double *J, double *dJ_dtab, double *dJ_dphi, double *dJ_df0);

/* orc_adj_run with Windkessel outlets (an extension): pressure iolet k with
 * wk_on[k] != 0 takes its density from a three-element model instead of its
 * table, wk[5k..5k+4] = (rho_ref, R1, C, R2, X0) (C >= 0): after the update
 * s -> s+1, whose outflow is Q,
 *   X(s+1) = X(s) + (Q - X/R2)/C (C > 0; no X/R2 term if R2 = 0), R2 Q (C = 0),
 *   rho_k(s+1) = rho_ref + R1 Q + X(s+1),  X(0) = X0, rho_k(0) = rho_ref + X0.
 * dJ_dtab of such an outlet is the derivative with respect to the density it
 * held at each step.  Returns -1 if a flagged iolet is not a pressure iolet
 * or has C < 0. */
int orc_adj_run_wk(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
                   const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
                   int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights, const int32_t *wk_on,
                   const double *wk, const double *f0, double *J, double *dJ_dtab, double *dJ_dphi,
                   double *dJ_df0);

/* Tangent-linear model (oracle_tangent.c): the derivative dJ of the
 * objective of orc_adj_run (same arguments) in the direction given by df0
 * [n*19] (perturbation of the initial state, may be NULL), dtab
 * [n_io][nsteps] (perturbation of the table value iolet k uses at step
 * t0+s, may be NULL) and dphi [n] (porosity perturbation, may be NULL).
 * Serial.  Returns 0, or -1 on a bad argument, link code or allocation
 * failure. */
int orc_tl_run(int64_t n, const int32_t *coords, const int32_t *nbr, double tau, double rho0,
               const orc_iolet *io, int32_t n_io, const double *phi, int64_t t0, int64_t nsteps,
               int64_t obj_t0, int64_t obj_t1, int32_t objective, const double *weights, const double *f0,
               const double *df0, const double *dtab, const double *dphi, double *dJ);

/* Number of OpenMP threads the oracle uses. */
int32_t orc_threads(void);
/* Use n > 0 OpenMP threads from now on (for timing). */
void orc_set_threads(int32_t n);

/* Sum of WSS over all sites with a wall link (compensated). */
double orc_wss_sum(int64_t n, const int32_t *nbr, double tau, const double *f);

#ifdef __cplusplus
}
#endif
#endif
