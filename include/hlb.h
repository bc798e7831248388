/*
 * hlb.h -- C ABI of the MI355X (gfx950) sparse D3Q19 lattice-Boltzmann
 * (LBGK) library.
 *
 * The method is the one of Zacharoudiou, McCullough and Coveney,
 * "Development and performance of a HemeLB GPU code for human-scale blood
 * flow simulation" (arXiv 2202.11770):
 *   - D3Q19 lattice and single-relaxation-time (BGK) collision, eq. (3a),
 *     followed by streaming, eq. (3b)                         (Sec. 2.2)
 *   - equilibrium eq. (4) (with the standard 1/2 factors on the
 *     second-order terms), moments eqs. (5)-(6)                (Sec. 2.2)
 *   - mid-link bounce-back at walls                            (Sec. 2.3.1)
 *   - velocity iolets by Ladd's corrected bounce-back and pressure iolets by
 *     a ghost density                                          (Sec. 2.3.2)
 *   - sites grouped by collision-streaming type, a wavefront-uniform code
 *     path per group, structure-of-arrays populations (per tile of 4096
 *     sites), f_old / f_new swapped by pointer each step     (Sec. 3.2.2-3.2.3)
 * computed on the GPU as a pull (gather-then-collide) update over a sparse
 * list of fluid sites, lexicographic within each group by default.
 *
 * Conventions (every function):
 *   - returns hlb_status: HLB_OK (0) or a negative error code; the text of
 *     the last failure on the calling thread is hlb_last_error().
 *   - inputs are caller-owned and copied before return; the context owns all
 *     device memory until hlb_destroy.
 *   - site-indexed arrays are in the CALLER's site order (the order of
 *     hlb_create's inputs), whatever order the library uses internally.
 *   - a context is not thread-safe; distinct contexts are independent.
 *   - host pointers are plain CPU memory; "device" pointers are GPU memory
 *     of the current HIP device (e.g. torch tensors' data_ptr()).
 *
 * Lattice conventions shared with every producer of inputs:
 *   velocity order, opposite directions adjacent (opp(i) = i+1 for odd i):
 *     0 (0,0,0)
 *     1 (+1,0,0)  2 (-1,0,0)  3 (0,+1,0)  4 (0,-1,0)  5 (0,0,+1)  6 (0,0,-1)
 *     7 (+1,+1,0) 8 (-1,-1,0) 9 (+1,-1,0) 10 (-1,+1,0)
 *     11 (+1,0,+1) 12 (-1,0,-1) 13 (+1,0,-1) 14 (-1,0,+1)
 *     15 (0,+1,+1) 16 (0,-1,-1) 17 (0,+1,-1) 18 (0,-1,+1)
 *   weights 1/3 (i=0), 1/18 (1-6), 1/36 (7-18); c_s^2 = 1/3; dx = dt = 1.
 */
#ifndef HLB_H
#define HLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hlb_ctx hlb_ctx; /* opaque, owned by the library */

typedef enum {
  HLB_OK = 0,
  HLB_EINVAL = -1,   /* invalid argument; nothing was changed */
  HLB_ENOMEM = -2,   /* device or host allocation failed, or above the budget */
  HLB_EDEVICE = -3,  /* a HIP runtime call failed */
  HLB_ESTATE = -4,   /* call not valid in the context's current state */
  HLB_ENUMERIC = -5  /* a non-finite value was found in the state */
} hlb_status;

/* Storage of the 19 populations.  FP64 stores f_i in double and collides in
 * double (the paper's variables); the shifted low-precision forms store the
 * deviation f_i - w_i rho0 from the rest state in float / IEEE half (round
 * to nearest even) and collide in float.  Mass-balance sums are FP64 in
 * every form. */
typedef enum { HLB_F64 = 0, HLB_F32_SHIFTED = 1, HLB_F16_SHIFTED = 2 } hlb_storage;

/* Site types (Sec. 3.2.2: the six collision-streaming types). */
enum {
  HLB_SITE_BULK = 0,
  HLB_SITE_WALL = 1,
  HLB_SITE_INLET = 2,
  HLB_SITE_OUTLET = 3,
  HLB_SITE_INLET_WALL = 4,
  HLB_SITE_OUTLET_WALL = 5
};

/* Neighbour-table codes: >= 0 a fluid site id, HLB_LINK_WALL a wall link,
 * -(2+k) a link through iolet k. */
#define HLB_LINK_WALL (-1)
#define HLB_LINK_IOLET(k) (-(2 + (k)))

/* Internal site order (all keep the six types grouped). */
typedef enum {
  HLB_ORDER_INPUT = 0,  /* caller order within each group */
  HLB_ORDER_LEX = 1,    /* lexicographic (z, y, x) */
  HLB_ORDER_MORTON = 2, /* Morton (Z-order) curve */
  HLB_ORDER_BRICK = 3,  /* Morton order of 4x4x4 bricks, lexicographic inside */
  HLB_ORDER_BANDS = 4,  /* bands of 2^order_block consecutive y rows, in y
                           order; lexicographic (z, y, x) inside a band
                           (default, 128 rows: the same as lexicographic
                           below 128 rows in y) */
  HLB_ORDER_COLUMNS = 5 /* columns of 2^order_block x 2^order_block in (x, y),
                           in (y, x) order; lexicographic (z, y, x) inside */
} hlb_order;

enum { HLB_IOLET_VELOCITY = 0, HLB_IOLET_PRESSURE = 1 };
enum { HLB_ROLE_INLET = 0, HLB_ROLE_OUTLET = 1 };

/* One inlet or outlet ("iolet", Sec. 2.3.2).
 * Velocity kind (Ladd): a population leaving site x along c_i through the
 * iolet comes back as f'_i - 6 w_i rho0 (c_i . U) (rho0 replaced by the
 * site's density at s with hlb_options.ladd_rho_local), U = A_k(s) W(m) v_k, with
 * m = x + c_i/2 the link midpoint, W(m) = max(0, 1 - d^2/R^2) where d is the
 * distance of m from the iolet axis (centre, normal) (W = 1 if radius <= 0),
 * and v_k = vdir (the normal if vdir is zero).
 * Pressure kind (ghost density): it comes back as the equilibrium at density
 * rho_k(s) and the site's velocity projected on the normal.
 * A_k(s) / rho_k(s) is the iolet's table at s mod len (hlb_set_iolet_table);
 * the update from time s to s+1 uses the value at s. */
typedef struct {
  int32_t kind;      /* HLB_IOLET_VELOCITY or HLB_IOLET_PRESSURE */
  int32_t role;      /* HLB_ROLE_INLET or HLB_ROLE_OUTLET (selects the site type) */
  double centre[3];  /* a point of the iolet plane, lattice units */
  double normal[3];  /* unit normal pointing into the fluid */
  double radius;     /* profile radius R; <= 0: uniform weight */
  double vdir[3];    /* direction of the imposed velocity; zero vector: normal */
} hlb_iolet;

typedef struct {
  int32_t storage;     /* hlb_storage (default HLB_F64) */
  int32_t order;       /* hlb_order (default HLB_ORDER_BANDS) */
  int32_t xcd_remap;   /* K > 0: renumber the bulk kernel's workgroups so that
                          each of the 8 XCDs gets K consecutive 256-position
                          blocks of every window of 8K blocks; 0: plain block
                          order; -1 (default): chosen by the library from the
                          storage and the buffer size (FP16 0; FP64 64, or 256
                          when a population buffer exceeds 4 GiB; FP32 8, or
                          128); hlb_info reports the value in use.  Results do
                          not depend on it. */
  int32_t adjoint;     /* 1: enable hlb_adjoint_run (FP64 storage, pull
                          scheme; its buffers are allocated at the first run);
                          default 0 */
  double rho0;         /* reference density (default 1.0) */
  int64_t max_device_bytes; /* 0: no limit; otherwise HLB_ENOMEM above it */
  int32_t scheme;      /* HLB_SCHEME_PULL (default) or HLB_SCHEME_PUSH */
  int32_t sites_per_thread; /* bulk+wall sites per GPU thread in the full pull
                               step: 1 or 2; 0 (default): the measured best
                               for the storage type.  Results do not depend
                               on it. */
  int32_t graph_steps; /* k > 0 (even, up to 4096): hlb_step replays a
                          captured HIP graph of k steps for as many whole
                          graphs as fit and launches the rest one by one;
                          0 (default): every step is its own launch.  A
                          graph is recaptured when a buffer, table pointer,
                          porosity or Windkessel setting changes; it is not
                          used while timing is on.  Results do not depend on
                          it (bit for bit, except where atomics already make
                          the Windkessel outflow order-dependent). */
  int32_t order_block; /* log2 of the band / column width of
                          HLB_ORDER_BANDS and HLB_ORDER_COLUMNS, 1..16
                          (default 7); ignored by the other orders */
  int32_t ladd_rho_local; /* density in the Ladd rule (Sec. 2.3.2):
                          0 (default) the reference density rho0;
                          1 the site's own density at the time of the
                          update (not with adjoint = 1) */
} hlb_options;

/* Order of the fused update (Sec. 3.2 implements push and names pull as
 * future work).  PULL: each site gathers its populations from its
 * neighbours' post-collision values, collides and stores the result (the
 * buffers hold post-collision states).  PUSH: each site collides its own
 * pre-collision state and scatters the results to the neighbours that
 * receive them (the buffers hold pre-collision states).  Both compute the
 * same update; hlb_adjoint_run needs PULL. */
enum { HLB_SCHEME_PULL = 0, HLB_SCHEME_PUSH = 1 };

/* Fill *opt with the defaults. */
hlb_status hlb_default_options(hlb_options *opt);

/* Create a simulation (Sec. 3.2.1: device set-up).
 *   n_sites   number of fluid sites, 1 <= n_sites < 2^30 - 2^13
 *   coords    [n][3] int32 lattice coordinates, each in [0, 2^20)
 *   site_type [n] uint8, HLB_SITE_*; must agree with the link codes
 *   nbr       [n][19] int32 push-direction table: nbr[x][i] = id of the site
 *             at coords[x] + c_i, HLB_LINK_WALL or HLB_LINK_IOLET(k);
 *             nbr[x][0] == x; must be symmetric
 *             (nbr[x][i] = y >= 0 implies nbr[y][opp(i)] = x)
 *   tau       relaxation time, > 1/2 (eq. (8): viscosity (tau - 1/2)/3)
 *   iolets    [n_iolets] descriptors (may be NULL if n_iolets == 0)
 *   opt       options or NULL for the defaults
 *   out       receives the context
 * The state starts at rest (f = f^eq(rho0, 0)) at time t = 0; velocity
 * tables start as {0}, pressure tables as {rho0}.
 * Errors: HLB_EINVAL (any rule above broken; message names the first
 * offending site/link), HLB_ENOMEM, HLB_EDEVICE. */
hlb_status hlb_create(int64_t n_sites, const int32_t *coords, const uint8_t *site_type,
                      const int32_t *nbr, double tau, const hlb_iolet *iolets, int32_t n_iolets,
                      const hlb_options *opt, hlb_ctx **out);

/* Release all device and host memory of the context (NULL is accepted). */
hlb_status hlb_destroy(hlb_ctx *ctx);

/* Run the context's work on a caller-owned HIP stream (hipStream_t); NULL
 * restores the context's own stream.  The stream must outlive its use. */
hlb_status hlb_set_stream(hlb_ctx *ctx, void *hip_stream);

/* Per-step table of iolet k: A_k(s) (velocity) or rho_k(s) (pressure),
 * value at step s = values[s mod len]; len >= 1, values finite (host). */
hlb_status hlb_set_iolet_table(hlb_ctx *ctx, int32_t k, const double *values, int64_t len);

/* Porosity phi in [0,1] per site (host, [n], caller order; read at sites
 * with wall links only): a wall link returns (1 - phi) f'_i + phi w_i rho0,
 * i.e. a fraction phi leaks to a reservoir at rest density.  NULL removes
 * the porosity (plain bounce-back).  Not a rule of the paper. */
hlb_status hlb_set_porosity(hlb_ctx *ctx, const double *phi);

/* Device-array forms of the two setters above, for callers whose parameters
 * live on the GPU (torch tensors):
 *   hlb_set_iolet_table_device: values is a device array of len doubles.
 *     The values are checked on the device (finite; > 0 for a pressure
 *     iolet; HLB_EINVAL otherwise, nothing changed).  If len equals the
 *     iolet's current table length (and no Windkessel model is on), they are
 *     copied device to device into the library's table, ordered on the
 *     context stream before later steps; otherwise the library's table
 *     layout is rebuilt, which reads the len values back to the host once.
 *   hlb_set_porosity_device: phi is a device array [n_sites] of doubles in
 *     caller order (NULL removes the porosity); checked on the device
 *     (every value in [0,1], HLB_EINVAL otherwise, nothing changed) and
 *     reordered into the library's positions by a kernel.
 * Both wait for the check's one-word verdict; the caller's array may be
 * reused once the call has returned. */
hlb_status hlb_set_iolet_table_device(hlb_ctx *ctx, int32_t k, const void *values, int64_t len);
hlb_status hlb_set_porosity_device(hlb_ctx *ctx, const void *phi);

/* Reset the state to f = f^eq(rho(x), u(x)) (Sec. 3.1, step 1) at time t0.
 * rho [n] and u [n][3] are host arrays in caller order, or NULL for rho0 and
 * zero velocity.  Resets the mass-balance bookkeeping. */
hlb_status hlb_init_equilibrium(hlb_ctx *ctx, const double *rho, const double *u, int64_t t0);

/* Advance n >= 0 steps (t -> t + n), asynchronously on the context stream.
 * Each step: pull-gather with boundary rules, then BGK collision, for all
 * site groups; then the f_old / f_new pointer swap. */
hlb_status hlb_step(hlb_ctx *ctx, int64_t n);

/* Density, velocity [n][3] and wall shear stress of the state at the
 * current time t (pre-collision populations), in caller order.  Any output
 * may be NULL.  Wall shear stress (not defined by the paper) is the
 * tangential part of the traction sigma n, sigma = -(1 - 1/(2 tau)) times
 * the non-equilibrium second moment, n the normalised sum of the site's
 * wall-link directions; 0 at sites without wall links.
 * hlb_macros: host outputs, synchronises.  hlb_macros_device: device
 * outputs (double), asynchronous on the context stream. */
hlb_status hlb_macros(hlb_ctx *ctx, double *rho, double *u, double *wss);
hlb_status hlb_macros_device(hlb_ctx *ctx, void *rho, void *u, void *wss);

/* Pre-collision populations f_i(x, t) as [n][19] FP64, caller order (host,
 * synchronises). */
hlb_status hlb_get_state(hlb_ctx *ctx, double *f);
/* Set f_i(x, t) (host [n][19] FP64, caller order) and the time t.  Resets
 * the mass-balance bookkeeping. */
hlb_status hlb_set_state(hlb_ctx *ctx, const double *f, int64_t t);

/* Total mass M(t) = sum_x sum_i f_i (FP64 reduction) and the balance
 * residual R(t) = M(t) - M(t0) - (mass added by the boundary rules since
 * t0), t0 the last (re)initialisation.  Synchronises.  HLB_ENUMERIC if M is
 * not finite. */
hlb_status hlb_mass_balance(hlb_ctx *ctx, double *mass, double *residual);

/* hlb_mass_balance for callers that cannot allocate device memory or wait
 * on the host (code under HIP graph capture, tight serving loops): writes
 * out[0] = M(t) and out[1] = R(t), bit for bit the values hlb_mass_balance
 * returns, to `out`, caller-owned device memory of 2 doubles, asynchronously
 * on the context stream.  It calls no hipMalloc / hipFree and does not
 * synchronise; the non-finite check of hlb_mass_balance is left to the
 * caller.  The reduction's partial sums go to a fixed array of 8,192
 * doubles (64 KiB) in device memory that every GPU the library runs on
 * holds until the process ends; each call overwrites the slots it reads, so
 * nothing is cleared between calls, and any site count is served (larger
 * states stride over the slots).  All calls on one GPU share that array:
 * calls that may overlap on one GPU (two streams, two threads) race and
 * must be ordered by the caller.  Errors: HLB_EINVAL (null ctx or out),
 * HLB_EDEVICE. */
hlb_status hlb_mass_balance_noalloc(hlb_ctx *ctx, void *out);

/* Current time step t. */
hlb_status hlb_time(const hlb_ctx *ctx, int64_t *t);

typedef struct {
  int64_t n_sites;          /* fluid sites */
  int64_t n_padded;         /* positions incl. padding: each group starts on a multiple of
                               256, the total is a multiple of 4096 (one storage tile) */
  int64_t group_sites[6];   /* sites per group: bulk+wall, inlet, outlet,
                               inlet+wall, outlet+wall, ghosts (partition) */
  int32_t storage;          /* hlb_storage */
  int32_t order;            /* hlb_order */
  double bytes_per_lup;     /* algorithmic HBM bytes per lattice-site update: 19
                               population loads + 19 stores + table_bytes_per_site */
  int64_t device_bytes;     /* device memory held by the context */
  double table_bytes_per_site; /* neighbour-table bytes read per site update */
  int64_t n_segments;       /* segments of the bulk+wall group's table */
  int64_t n_iolets;         /* iolets given to hlb_create */
  int32_t adjoint;          /* hlb_adjoint_run enabled (opt.adjoint) */
  int32_t porous;           /* a porosity field is set */
  int32_t scheme;           /* hlb_scheme of the context */
  int32_t sites_per_thread; /* bulk+wall sites per thread of the full pull step */
  int32_t graph_steps;      /* steps per replayed graph in hlb_step (0: none) */
  int32_t xcd_remap;        /* workgroup-to-XCD chunk in use (hlb_options.xcd_remap) */
} hlb_info_t;
hlb_status hlb_info(const hlb_ctx *ctx, hlb_info_t *info);

/* Kernel timing (HIP events on the context stream around each launch of the
 * step kernel, and around each reverse step of hlb_adjoint_run) while
 * enabled; hlb_stats reports the steps timed, the mean duration of the step
 * kernel and the mean stream time per step, and the same for the reverse
 * steps, in milliseconds.  Enabling or disabling resets the counts. */
hlb_status hlb_set_timing(hlb_ctx *ctx, int32_t enable);
typedef struct {
  int64_t steps;     /* steps timed since timing was enabled */
  double kernel_ms;  /* mean duration of one step kernel (all site groups) */
  double step_ms;    /* mean stream time per step, first to last timed event */
  int64_t adj_steps; /* reverse steps of hlb_adjoint_run timed */
  double adj_ms;     /* mean duration of one reverse step (both adjoint kernels) */
  double mlups;      /* million lattice-site updates per second over step_ms
                        (eq. (9): updated sites / step_ms); 0 if none timed */
  double alg_gbs;    /* algorithmic HBM GB/s of the step kernel: bytes_per_lup
                        (hlb_info_t) x updated sites / kernel_ms; 0 if none timed */
} hlb_stats_t;
hlb_status hlb_stats(hlb_ctx *ctx, hlb_stats_t *stats);

/* Windkessel outlet (not a rule of the paper; its outlook names resistance
 * and physiological outlets): pressure iolet k takes its ghost density from
 * a three-element model driven by its outflow Q_k(s) (net mass leaving
 * through the iolet's links during the update s -> s+1, as in
 * HLB_OBJ_IOLET_FLUX), in lattice density units:
 *   rho_k(s+1) = rho_ref + R1 Q_k(s) + X(s+1),
 *   X(s+1) = X(s) + (Q_k(s) - X(s)/R2) / C   if C > 0 (no leak term if R2 = 0),
 *   X(s+1) = R2 Q_k(s)                       if C = 0 (resistance R1 + R2).
 * Each update's outflow is accumulated in FP64 by the step kernel and the
 * state advanced by one small kernel after it.  rho_k starts at rho_ref + X0.
 * w = NULL turns the model off (the iolet keeps its last table);
 * hlb_set_iolet_table on the iolet also turns it off.  R1, C, R2 >= 0 and,
 * if C > 0 and R2 > 0, R2 C >= 1.  Not on a partition.  hlb_adjoint_run
 * carries the model through its sweeps (its checkpoints hold the model's
 * state).
 * hlb_windkessel_state: the density the next update uses, X and the last
 * update's outflow (synchronises).  State files and snapshots do not
 * include the model's state. */
typedef struct {
  double rho_ref, R1, C, R2, X0;
} hlb_windkessel;
hlb_status hlb_set_windkessel(hlb_ctx *ctx, int32_t k, const hlb_windkessel *w);
hlb_status hlb_windkessel_state(hlb_ctx *ctx, int32_t k, double *rho_next, double *X, double *Q_last);

/* ---- Domain split (Sec. 3.1's edge / mid-domain split with the halo
 * exchange of Sec. 3.2.3; pull order): one context per partition, the
 * exchange between them left to the caller (a device copy between two
 * contexts on one GPU, or RCCL send/recv between GPUs). ----
 *
 * hlb_create_part: as hlb_create, with a role per site:
 *   HLB_PART_MID   an owned site no other partition reads;
 *   HLB_PART_EDGE  an owned site whose populations another partition reads;
 *   HLB_PART_GHOST a copy of another partition's site that owned sites pull
 *                  from: only nbr[x][0] == x and its coordinates are used
 *                  (its links and type are ignored); it is never updated,
 *                  and macros, mass and state export skip it (its entries
 *                  of caller-order outputs are unspecified).
 * Owned sites' links may point at ghosts (no symmetry required there).  The
 * edge sites lead the bulk+wall group so that they can be updated first.
 * Needs the pull scheme and no adjoint.  Ghosts start as zero: exchange once
 * (hlb_halo_pack, transfer, hlb_halo_unpack) after init or set_state. */
enum { HLB_PART_MID = 0, HLB_PART_EDGE = 1, HLB_PART_GHOST = 2 };
hlb_status hlb_create_part(int64_t n_sites, const int32_t *coords, const uint8_t *site_type, const int32_t *nbr,
                           double tau, const hlb_iolet *iolets, int32_t n_iolets, const hlb_options *opt,
                           const uint8_t *role, hlb_ctx **out);

/* The halo lists (host, caller ids and directions 0..18): send entry k is
 * population send_dir[k] of edge site send_site[k]; receive entry k is
 * population recv_dir[k] of ghost site recv_site[k].  The peer's send list
 * must list the same (site, direction) pairs in the same order as this
 * receive list.  send_buf / recv_buf: the caller's device buffers of at
 * least n_send / n_recv values of the storage type, used by every later
 * pack and unpack (they must stay valid).  Errors: HLB_EINVAL (a send site
 * not EDGE, a receive site not GHOST, direction out of range, a missing
 * buffer), HLB_ESTATE (not a partition). */
hlb_status hlb_halo_set(hlb_ctx *ctx, int64_t n_send, const int32_t *send_site, const int32_t *send_dir,
                        void *send_buf, int64_t n_recv, const int32_t *recv_site, const int32_t *recv_dir,
                        void *recv_buf);
/* Pack the current state's send values into the send buffer / write the
 * receive buffer into the current state's ghost slots (context stream). */
hlb_status hlb_halo_pack(hlb_ctx *ctx);
hlb_status hlb_halo_unpack(hlb_ctx *ctx);
/* Direct exchange (the design for more than one GPU: the receiver's ghost
 * slots are written by the sender, no receive buffer and no unpack):
 * hlb_halo_ghost_slots: for n (ghost site, direction) pairs of a partition
 *   (host, caller ids), elem[k] (host, [n]) receives the element index of
 *   that ghost slot in the partition's population buffers (the same in
 *   both) and buf[0], buf[1] the two buffers' device addresses (fixed for
 *   the context's life).  Errors: HLB_EINVAL (not a ghost site, direction
 *   out of range, null output), HLB_ESTATE (not a partition).
 * hlb_halo_add_peer: adds a peer to which this partition sends n values:
 *   entry k is population dir[k] of edge site site[k] (host, caller ids),
 *   written to element peer_elem[k] (host) of the peer's buffers
 *   (peer_buf0, peer_buf1, device memory; from hlb_halo_ghost_slots, or
 *   the same buffers mapped from another GPU).  hlb_step_edge then writes
 *   the new values into the peer buffer with the index of the buffer it
 *   writes itself, and hlb_halo_pack the current values into the peer
 *   buffer with the index of its current one: the partitions must advance
 *   in lockstep from a common start (equal buffer indices), and a
 *   partition's hlb_step_edge must not start before its peers' previous
 *   hlb_step_edge has finished (the last reader of the slots it writes and
 *   the writer of those it reads); hlb_halo_unpack has nothing to do for
 *   such a peer.  Errors: HLB_EINVAL (n < 1, not an edge site, direction
 *   out of range, a negative element, null buffer), HLB_ESTATE.
 * hlb_halo_clear_peers: removes every peer. */
hlb_status hlb_halo_ghost_slots(hlb_ctx *ctx, int64_t n, const int32_t *site, const int32_t *dir, int64_t *elem,
                                void **buf);
hlb_status hlb_halo_add_peer(hlb_ctx *ctx, int64_t n, const int32_t *site, const int32_t *dir, void *peer_buf0,
                             void *peer_buf1, const int64_t *peer_elem);
hlb_status hlb_halo_clear_peers(hlb_ctx *ctx);
/* One step t -> t+1 in two launches, so that the transfer of the edge
 * values overlaps the rest of the update:
 *   hlb_step_edge: the iolet groups and the edge blocks of the bulk+wall
 *     group, then the pack of the new edge values into the send buffer;
 *   hlb_step_mid: the remaining blocks; then t advances.
 * The caller moves the peer's send buffer into this receive buffer once the
 * peer's hlb_step_edge has run (an event on the peer's stream), and calls
 * hlb_halo_unpack after hlb_step_mid, before the next step.  Between the two
 * calls only the transfer may touch the context (HLB_ESTATE otherwise). */
hlb_status hlb_step_edge(hlb_ctx *ctx);
hlb_status hlb_step_mid(hlb_ctx *ctx);

/* Run hlb_step_mid on a second caller-owned HIP stream (hipStream_t), so
 * that the mid-domain update of step t overlaps the edge update and the
 * exchange of the same step (Sec. 3.1: the edge sites are updated and sent
 * while the mid-domain sites are updated); NULL (the default) runs it on
 * the context's stream.  The library then orders nothing between the two
 * streams; the caller must make
 *   the context's stream wait for the previous hlb_step_mid before each
 *     hlb_step_edge (the mid step writes the sites the edge step reads and
 *     reads the buffer the edge step writes), and before any other call on
 *     the context;
 *   this stream wait for the previous hlb_step_edge (and for the work that
 *     set up the state) before each hlb_step_mid.
 * The stream must outlive its use.  Errors: HLB_ESTATE (between
 * hlb_step_edge and hlb_step_mid). */
hlb_status hlb_set_mid_stream(hlb_ctx *ctx, void *hip_stream);

/* Objective of hlb_adjoint_run (not a rule of the paper).
 *   HLB_OBJ_WSS (default): the wall shear stress (hlb_macros' definition)
 *     of the state at t, summed over the sites with wall links;
 *   HLB_OBJ_IOLET_FLUX: sum_k weights[k] Q_k(t), Q_k(t) the net outflow
 *     through iolet k during the update t-1 -> t: over the iolet's links,
 *     the post-collision population that leaves minus the one the iolet
 *     returns (with weight 1 on every iolet and no porosity, the mass the
 *     step loses).
 * weights: host, [n_iolets], copied; ignored (may be NULL) for HLB_OBJ_WSS.
 * Errors: HLB_EINVAL (unknown kind, weights NULL or not finite). */
enum { HLB_OBJ_WSS = 0, HLB_OBJ_IOLET_FLUX = 1 };
hlb_status hlb_set_objective(hlb_ctx *ctx, int32_t kind, const double *weights);

/* Differentiation (not a rule of the paper): the adjoint of the update.
 * From the current state at time t0, run n >= 1 steps and the reverse-time
 * sweep for the objective (hlb_set_objective)
 *   J = sum over t in (obj_t0, obj_t1], t0 < t <= t0 + n, of the objective
 *       at t,
 * with respect to
 *   dJ_dA   [n_iolets][n] (host, may be NULL): the table value iolet k uses
 *           in the update t0+s -> t0+s+1: the amplitude A_k(t0 + s) of a
 *           velocity iolet, the ghost density rho_k(t0 + s) of a pressure
 *           iolet (of a Windkessel outlet: the density its model gave it
 *           for that update, the model's later response to it included);
 *   dJ_dphi [n_sites] (host, caller order, may be NULL): each site's
 *           porosity (hlb_set_porosity), zero at sites without wall links,
 *           evaluated at the current porosity (0 if none is set).
 * The forward states are recomputed from n_snap device snapshots
 * (1 <= n_snap <= 4096, the start state's included; binomial checkpointing
 * after Griewank & Walther): the schedule takes the fewest forward steps
 * possible with n_snap slots, r n - C(n_snap + r, r - 1) with r the least
 * integer with C(n_snap + r, n_snap) >= n (hlb_revolve_forward_steps).
 * *forward_steps (may be NULL) receives the forward steps run.  The state
 * is left as it was (time t0).  Needs opt.adjoint at creation and FP64
 * storage (HLB_ESTATE otherwise). */
hlb_status hlb_adjoint_run(hlb_ctx *ctx, int64_t n, int64_t obj_t0, int64_t obj_t1, int32_t n_snap,
                           double *J, double *dJ_dA, double *dJ_dphi, int64_t *forward_steps);

/* hlb_adjoint_run with device outputs (doubles in GPU memory: J [1],
 * dJ_dA [n_iolets][n], dJ_dphi [n_sites] in caller order; dJ_dA and dJ_dphi
 * may be NULL), written asynchronously on the context stream: nothing is
 * read back to the host and the call does not wait for the sweep.  The
 * objective's finiteness is not checked (the caller reads J).
 * *forward_steps (host, may be NULL) is known when the call returns.  The
 * outputs come from the same kernels as those of hlb_adjoint_run: dJ_dphi
 * is bit for bit the same; J and dJ_dA, which are summed with atomics
 * (the iolet terms), can differ in the last bits, as between two runs of
 * either call. */
hlb_status hlb_adjoint_run_device(hlb_ctx *ctx, int64_t n, int64_t obj_t0, int64_t obj_t1, int32_t n_snap,
                                  void *J, void *dJ_dA, void *dJ_dphi, int64_t *forward_steps);

/* Forward steps hlb_adjoint_run takes for n >= 1 steps with n_snap
 * snapshots (1 <= n_snap <= 4096), without running anything: for planning
 * snapshot memory (n_snap state buffers) against recomputation.  Host-only;
 * needs no context or device.  Errors: HLB_EINVAL (arguments out of range,
 * steps NULL). */
hlb_status hlb_revolve_forward_steps(int64_t n, int32_t n_snap, int64_t *steps);

/* Device snapshots of the whole state (for checkpointing schedules).
 * hlb_snapshot_alloc reserves n_slots slots (frees previous ones). */
hlb_status hlb_snapshot_alloc(hlb_ctx *ctx, int32_t n_slots);
hlb_status hlb_snapshot_save(hlb_ctx *ctx, int32_t slot);
hlb_status hlb_snapshot_restore(hlb_ctx *ctx, int32_t slot);

/* Bit-exact host copy of the state (both population buffers, time and
 * bookkeeping): hlb_state_bytes gives the size; save writes it to host
 * memory, load restores it.  Synchronise. */
hlb_status hlb_state_bytes(const hlb_ctx *ctx, int64_t *bytes);
hlb_status hlb_state_save(hlb_ctx *ctx, void *host_buf);
hlb_status hlb_state_load(hlb_ctx *ctx, const void *host_buf);

/* Wait for all work queued on the context stream. */
hlb_status hlb_sync(hlb_ctx *ctx);

/* Measurement aid, not part of the method: bandwidth in GB/s (read + write
 * bytes over time) of a plain non-temporal device-to-device copy of `bytes`
 * (>= 1 MiB, multiple of 16) repeated `reps` times on the null stream of the
 * current device -- the practical ceiling for the step kernel.  Allocates and
 * frees two buffers of `bytes`. */
hlb_status hlb_copy_bandwidth(int64_t bytes, int32_t reps, double *gbs);

/* Message of the last failure on this thread ("" if none). */
const char *hlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HLB_H */
