// Host runtime of the C ABI in hlb.h: input validation, grouping of sites by
// collision-streaming type, space-filling-curve ordering, construction of
// the pull neighbour table and iolet link coefficients, device memory, time
// bookkeeping, snapshots and error reporting.  All arithmetic of the update
// itself is in hlb_kernels.hip.

#include <hip/hip_runtime.h>
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "hlb.h"
#include "hlb_adjoint.h"
#include "hlb_aux.h"
#include "hlb_halo.h"
#include "hlb_internal.h"
#include "hlb_noalloc.h"

using namespace hlb;

namespace {

thread_local std::string g_err;

hlb_status fail(hlb_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      if (e_ == hipErrorOutOfMemory) return fail(HLB_ENOMEM, "%s: %s", #call, hipGetErrorString(e_)); \
      return fail(HLB_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));                    \
    }                                                                                      \
  } while (0)

constexpr int Q = 19;
// Velocity set of the input convention (hlb.h), host copy for table building.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
inline int OPP(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
inline double W(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

size_t storage_bytes(int storage) {
  return storage == HLB_F64 ? 8 : (storage == HLB_F32_SHIFTED ? 4 : 2);
}

// Workgroup-to-XCD chunk of the step kernel when the caller leaves it to
// the library (hlb_options.xcd_remap = -1), from sweeps of the chunk (0 to
// 4096 blocks) on the 2e7- and 2e8-site trees: FP16 runs fastest in plain
// block order at both sizes; FP64 with 64 blocks per chunk while a
// population buffer fits in 4 GiB and 256 above; FP32 with 8 and 128.
int auto_xcd_chunk(int storage, int64_t np) {
  const bool big = (uint64_t)Q * (uint64_t)np * storage_bytes(storage) > (uint64_t(1) << 32);
  if (storage == HLB_F16_SHIFTED) return 0;
  if (storage == HLB_F32_SHIFTED) return big ? 128 : 8;
  return big ? 256 : 64;
}

// group of a site type: bulk and wall are merged (Sec. 3.2.2)
inline int group_of(int type) {
  switch (type) {
    case HLB_SITE_BULK:
    case HLB_SITE_WALL: return 0;
    case HLB_SITE_INLET: return 1;
    case HLB_SITE_OUTLET: return 2;
    case HLB_SITE_INLET_WALL: return 3;
    case HLB_SITE_OUTLET_WALL: return 4;
    default: return -1;
  }
}

inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | v << 32) & 0x1f00000000ffffull;
  v = (v | v << 16) & 0x1f0000ff0000ffull;
  v = (v | v << 8) & 0x100f00f00f00f00full;
  v = (v | v << 4) & 0x10c30c30c30c30c3ull;
  v = (v | v << 2) & 0x1249249249249249ull;
  return v;
}
inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | spread3(y) << 1 | spread3(z) << 2; }

// Extent of the coordinates (max + 1 per axis) and the block width 2^b of
// the band and column orders.
struct KeyGeom {
  uint64_t nx = 1, ny = 1, nz = 1;
  int b = 6;
};

// Sort key of a site.  Every key stays below 2^63 (coordinates < 2^20; the
// mixed-radix keys below are at most about nx ny nz (1 + 2^-b)^2).
uint64_t sfc_key(int order, int64_t id, const int32_t *c, const KeyGeom &kg) {
  const uint64_t x = (uint64_t)c[0], y = (uint64_t)c[1], z = (uint64_t)c[2];
  const uint64_t B = uint64_t(1) << kg.b, m = B - 1;
  switch (order) {
    case HLB_ORDER_LEX: return z << 40 | y << 20 | x;
    case HLB_ORDER_MORTON: return morton(x, y, z);
    case HLB_ORDER_BRICK: return morton(x >> 2, y >> 2, z >> 2) << 6 | (z & 3) << 4 | (y & 3) << 2 | (x & 3);
    case HLB_ORDER_BANDS:  // bands of B rows in y, (z, y, x) inside
      return ((y >> kg.b) * kg.nz + z) * (B * kg.nx) + (y & m) * kg.nx + x;
    case HLB_ORDER_COLUMNS: {  // B x B columns in (x, y), (z, y, x) inside
      const uint64_t nxb = (kg.nx + m) >> kg.b;
      return (((y >> kg.b) * nxb + (x >> kg.b)) * kg.nz + z) * (B * B) + (y & m) * B + (x & m);
    }
    default: return (uint64_t)id;
  }
}

using KeyId = std::pair<uint64_t, int32_t>;

void psort(std::vector<KeyId> &v) {
  const size_t n = v.size();
  const int T = omp_get_max_threads();
  if (n < (1u << 16) || T == 1) {
    std::sort(v.begin(), v.end());
    return;
  }
  std::vector<size_t> cut(T + 1);
  for (int t = 0; t <= T; ++t) cut[t] = n * (size_t)t / (size_t)T;
#pragma omp parallel for schedule(static, 1)
  for (int t = 0; t < T; ++t) std::sort(v.begin() + cut[t], v.begin() + cut[t + 1]);
  for (int w = 1; w < T; w *= 2) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < T; t += 2 * w) {
      if (t + w < T) std::inplace_merge(v.begin() + cut[t], v.begin() + cut[t + w], v.begin() + cut[std::min(t + 2 * w, T)]);
    }
  }
}

struct TimedStep {
  hipEvent_t e[2];
};

// Everything a captured step graph bakes into its kernel arguments: a graph
// is replayed only while all of it is unchanged.
bool same_launch(const DevPtrs &a, const DevPtrs &b) {
  return a.f[0] == b.f[0] && a.f[1] == b.f[1] && a.seg_off == b.seg_off && a.seg_base == b.seg_base &&
         a.seg_delta == b.seg_delta && a.nbr_io == b.nbr_io && a.order == b.order && a.corr == b.corr &&
         a.io == b.io && a.tables == b.tables && a.phi == b.phi && a.acc == b.acc && a.wk_rho == b.wk_rho &&
         a.io_flux == b.io_flux && a.wk == b.wk;
}
bool same_launch(const LaunchCfg &a, const LaunchCfg &b) {
  return a.storage == b.storage && a.tau == b.tau && a.rho0 == b.rho0 && a.xcd_chunk == b.xcd_chunk &&
         a.porous == b.porous && a.scheme == b.scheme && a.sites_per_thread == b.sites_per_thread &&
         a.ladd_local == b.ladd_local;
}

}  // namespace

struct hlb_ctx {
  Layout L;
  DevPtrs d;
  LaunchCfg cfg;
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t mid_stream = nullptr;  // hlb_step_mid's stream (null: stream)
  int cur = 0;          // buffer holding the post-collision state of time t
  bool direct = true;   // other buffer holds the pre-collision state of t
  // partition (hlb_create_part): per-site role and caller id -> position
  std::vector<uint8_t> role_host;
  std::vector<int32_t> inv_host;
  struct Halo {
    int32_t *send_pos = nullptr, *send_dir = nullptr, *recv_pos = nullptr, *recv_dir = nullptr;
    void *send_buf = nullptr, *recv_buf = nullptr;  // caller's device buffers
    int64_t n_send = 0, n_recv = 0;
    bool defined = false;
    int64_t bytes = 0;
  } halo;
  // direct exchange (hlb_halo_add_peer): values written straight into peer
  // partitions' ghost slots
  struct Peer {
    int32_t *pos = nullptr, *dir = nullptr;  // this partition's positions and directions
    int64_t *elem = nullptr;                 // the peer's element indices
    int64_t n = 0;
    void *buf[2] = {nullptr, nullptr};       // the peer's population buffers
    int64_t bytes = 0;
  };
  std::vector<Peer> peers;
  bool split_pending = false;  // hlb_step_edge done, hlb_step_mid due
  bool adj_on = false;         // opt.adjoint at creation
  // Windkessel outlets (hlb_set_windkessel)
  std::vector<int32_t> wk_on;
  int n_wk = 0;
  int64_t t = 0;
  int64_t t0 = 0;       // last (re)initialisation
  double m0 = 0.0;      // mass at t0
  int order = HLB_ORDER_LEX;
  int64_t max_bytes = 0;
  int64_t dev_bytes = 0;
  int64_t staging_len = 0;             // doubles in d.io_scratch
  int64_t table_bytes = 0;             // device bytes of the pull tables
  std::vector<int32_t> order_host;     // [np] caller id per position
  std::vector<hlb_iolet> iolets;
  std::vector<std::vector<double>> tables;
  int64_t tables_len = 0;              // doubles in d.tables
  std::vector<int64_t> tab_off;        // offset of each iolet's table in d.tables
  std::vector<uint8_t> tab_dev;        // 1: d.tables holds a newer table than `tables` (device setter)
  int32_t *flag_dev = nullptr;         // [1] result of the checks of caller device arrays
  // timing
  bool timing = false;
  std::vector<TimedStep> pool;
  size_t n_timed = 0;
  int64_t steps_timed = 0;
  double sum_kernel = 0, sum_step = 0;
  std::vector<TimedStep> adj_pool;  // events around the adjoint step kernels
  size_t n_adj_timed = 0;
  int64_t adj_steps_timed = 0;
  double sum_adj = 0;
  // snapshots
  struct Snap {
    void *f[2] = {nullptr, nullptr};
    double *acc = nullptr;
    int64_t t = 0, t0 = 0;
    double m0 = 0;
    int cur = 0;
    bool direct = true;
    bool valid = false;
  };
  std::vector<Snap> snaps;
  // adjoint
  AdjBuffers adj;
  int64_t adj_dA_len = 0;
  std::vector<void *> adj_slots;  // checkpoint buffers (post-collision state)
  // the Windkessel outlets' state per checkpoint slot: WkParams [n_iolets]
  // then the densities [n_iolets][2]
  void *adj_wk_slots = nullptr;
  int64_t adj_wk_nslots = 0;
  // replayed step graphs (hlb_step): one per starting buffer, captured with
  // the time read from t_dev
  int graph_steps = 0;            // steps per graph; 0: no graphs
  int64_t *t_dev = nullptr;       // [1] time at the start of the next replay
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  DevPtrs graph_d;                // what the graphs were captured with
  LaunchCfg graph_cfg;
  int graph_nwk = -1;
};

namespace {

size_t buf_bytes(const hlb_ctx *c) { return (size_t)Q * (size_t)c->L.np * storage_bytes(c->cfg.storage); }

hlb_status dev_alloc(hlb_ctx *c, void **p, size_t bytes) {
  if (c->max_bytes > 0 && c->dev_bytes + (int64_t)bytes > c->max_bytes)
    return fail(HLB_ENOMEM, "device budget of %lld bytes exceeded (need %lld more)", (long long)c->max_bytes,
                (long long)bytes);
  hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(HLB_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  c->dev_bytes += (int64_t)bytes;
  return HLB_OK;
}

void free_halo(hlb_ctx *c) {
  auto F = [](void *p) { if (p) (void)hipFree(p); };
  F(c->halo.send_pos); F(c->halo.send_dir); F(c->halo.recv_pos); F(c->halo.recv_dir);
  c->dev_bytes -= c->halo.bytes;
  c->halo = hlb_ctx::Halo();
}

void free_peers(hlb_ctx *c) {
  for (auto &q : c->peers) {
    if (q.pos) (void)hipFree(q.pos);
    if (q.dir) (void)hipFree(q.dir);
    if (q.elem) (void)hipFree(q.elem);
    c->dev_bytes -= q.bytes;
  }
  c->peers.clear();
}

void free_all(hlb_ctx *c) {
  free_halo(c);
  free_peers(c);
  auto F = [](void *p) { if (p) (void)hipFree(p); };
  F(c->d.f[0]); F(c->d.f[1]); F(c->d.nbr_io); F(c->d.seg_off); F(c->d.seg_base); F(c->d.seg_delta); F(c->d.order); F(c->d.corr); F(c->d.io); F(c->d.tables);
  F(c->d.phi); F(c->d.acc); F(c->d.partial); F(c->d.io_scratch);
  F(c->d.wk_rho); F(c->d.io_flux); F(c->d.wk);
  F(c->flag_dev);
  c->flag_dev = nullptr;
  for (auto &s : c->snaps) { F(s.f[0]); F(s.f[1]); F(s.acc); }
  c->snaps.clear();
  F(c->adj.mu); F(c->adj.nu); F(c->adj.J); F(c->adj.dA); F(c->adj.dphi); F(c->adj.w); F(c->adj.blist);
  for (void *q : c->adj_slots) F(q);
  c->adj_slots.clear();
  F(c->adj_wk_slots);
  c->adj_wk_slots = nullptr;
  c->adj_wk_nslots = 0;
  F(c->adj.wq); F(c->adj.lamX);
  c->adj = AdjBuffers();
  for (auto &ts : c->pool)
    for (auto &e : ts.e) (void)hipEventDestroy(e);
  for (auto &ts : c->adj_pool)
    for (auto &e : ts.e) (void)hipEventDestroy(e);
  c->adj_pool.clear();
  c->pool.clear();
  for (auto &g : c->graph)
    if (g) (void)hipGraphExecDestroy(g);
  c->graph[0] = c->graph[1] = nullptr;
  F(c->t_dev);
  c->t_dev = nullptr;
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  c->d = DevPtrs();
}

hlb_status upload_tables(hlb_ctx *c) {
  const int K = (int)c->iolets.size();
  if (K == 0) return HLB_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  // tables last set from device memory live only in d.tables: fetch them
  // before the concatenation is rebuilt
  for (int k = 0; k < K && k < (int)c->tab_dev.size(); ++k)
    if (c->tab_dev[k]) {
      HIP_TRY(hipMemcpy(c->tables[k].data(), c->d.tables + c->tab_off[k], c->tables[k].size() * sizeof(double),
                        hipMemcpyDeviceToHost));
      c->tab_dev[k] = 0;
    }
  c->tab_off.assign(K, 0);
  c->tab_dev.assign(K, 0);
  std::vector<IoletDev> io(K);
  std::vector<double> all;
  for (int k = 0; k < K; ++k) {
    io[k].kind = c->iolets[k].kind;
    io[k].tab_len = (int32_t)c->tables[k].size();
    io[k].tab_off = (int64_t)all.size();
    c->tab_off[k] = io[k].tab_off;
    for (int a = 0; a < 3; ++a) io[k].n[a] = c->iolets[k].normal[a];
    io[k].wk = k < (int)c->wk_on.size() ? c->wk_on[k] : 0;
    io[k].pad = 0;
    all.insert(all.end(), c->tables[k].begin(), c->tables[k].end());
  }
  if (c->d.tables) {
    (void)hipFree(c->d.tables);
    c->d.tables = nullptr;
    c->dev_bytes -= c->tables_len * (int64_t)sizeof(double);
    c->tables_len = 0;
  }
  void *p = nullptr;
  hlb_status st = dev_alloc(c, &p, all.size() * sizeof(double));
  if (st) return st;
  c->d.tables = static_cast<double *>(p);
  c->tables_len = (int64_t)all.size();
  HIP_TRY(hipMemcpy(c->d.tables, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice));
  if (!c->d.io) {
    st = dev_alloc(c, &p, K * sizeof(IoletDev));
    if (st) return st;
    c->d.io = static_cast<IoletDev *>(p);
  }
  HIP_TRY(hipMemcpy(c->d.io, io.data(), K * sizeof(IoletDev), hipMemcpyHostToDevice));
  return HLB_OK;
}

// Mass of the stored zero: N rho0 for the shifted forms (sum_i w_i = 1),
// 0 for FP64, which stores f itself.
double mass_offset(const hlb_ctx *c) {
  // the shift sums to rho0 per owned site (ghosts hold no mass of their own)
  return c->cfg.storage == HLB_F64 ? 0.0 : (double)(c->L.n_sites - c->L.n_ghost) * c->cfg.rho0;
}

hlb_status check_ctx(const hlb_ctx *c) {
  if (!c) return fail(HLB_EINVAL, "null context");
  return HLB_OK;
}

hlb_status bind(hlb_ctx *c) {
  HIP_TRY(hipSetDevice(c->device));
  return HLB_OK;
}

hlb_status compute_mass(hlb_ctx *c, double *sum_g) {
  HIP_TRY(launch_mass(c->cfg, c->L, c->d, c->cur, c->stream));
  HIP_TRY(hipMemcpyAsync(sum_g, c->d.partial, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HLB_OK;
}

hlb_status reset_balance(hlb_ctx *c) {
  HIP_TRY(launch_zero(c->d.acc, 4, c->stream));
  double s = 0;
  hlb_status st = compute_mass(c, &s);
  if (st) return st;
  c->m0 = mass_offset(c) + s;
  c->t0 = c->t;
  return HLB_OK;
}

// Device staging for host exchanges, grown to `doubles` on demand.
hlb_status ensure_staging(hlb_ctx *c, int64_t doubles) {
  if (c->staging_len >= doubles) return HLB_OK;
  if (c->d.io_scratch) {
    (void)hipFree(c->d.io_scratch);
    c->dev_bytes -= c->staging_len * (int64_t)sizeof(double);
    c->d.io_scratch = nullptr;
    c->staging_len = 0;
  }
  void *p = nullptr;
  hlb_status st = dev_alloc(c, &p, (size_t)doubles * sizeof(double));
  if (st) return st;
  c->d.io_scratch = static_cast<double *>(p);
  c->staging_len = doubles;
  return HLB_OK;
}

// Runs launch_check_values on a caller's device array and waits for the
// verdict: HLB_OK if every value keeps the rule, HLB_EINVAL (with `what`
// in the message) if one does not.
hlb_status check_device_values(hlb_ctx *c, const double *v, int64_t n, int mode, const char *what) {
  if (!c->flag_dev) {
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, sizeof(int32_t))) return st;
    c->flag_dev = static_cast<int32_t *>(p);
  }
  HIP_TRY(launch_check_values(v, n, mode, c->flag_dev, c->stream));
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, c->flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (bad) return fail(HLB_EINVAL, "%s", what);
  return HLB_OK;
}

}  // namespace

extern "C" {

const char *hlb_last_error(void) { return g_err.c_str(); }

hlb_status hlb_default_options(hlb_options *opt) {
  if (!opt) return fail(HLB_EINVAL, "null options");
  opt->storage = HLB_F64;
  opt->order = HLB_ORDER_BANDS;
  opt->xcd_remap = -1;
  opt->adjoint = 0;
  opt->rho0 = 1.0;
  opt->max_device_bytes = 0;
  opt->scheme = HLB_SCHEME_PULL;
  opt->sites_per_thread = 0;
  opt->graph_steps = 0;
  opt->order_block = 7;
  opt->ladd_rho_local = 0;
  return HLB_OK;
}

static hlb_status create_impl(int64_t n, const int32_t *coords, const uint8_t *type, const int32_t *nbr, double tau,
                              const hlb_iolet *iolets, int32_t n_iolets, const hlb_options *opt_in, const uint8_t *role,
                              hlb_ctx **out) {
  g_err.clear();
  if (!out) return fail(HLB_EINVAL, "out is null");
  *out = nullptr;
  if (!coords || !type || !nbr) return fail(HLB_EINVAL, "coords, site_type and nbr must be non-null");
  // positions (padding included) stay below 2^30, so that a position plus or
  // minus np fits in int32 in the kernels
  if (n < 1 || n >= (int64_t)(1 << 30) - 8192) return fail(HLB_EINVAL, "n_sites=%lld out of range", (long long)n);
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(HLB_EINVAL, "tau=%g must be finite and > 1/2", tau);
  if (n_iolets < 0 || (n_iolets > 0 && !iolets)) return fail(HLB_EINVAL, "bad iolet list");
  hlb_options opt;
  hlb_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.storage < HLB_F64 || opt.storage > HLB_F16_SHIFTED) return fail(HLB_EINVAL, "bad storage %d", opt.storage);
  if (opt.order < HLB_ORDER_INPUT || opt.order > HLB_ORDER_COLUMNS) return fail(HLB_EINVAL, "bad order %d", opt.order);
  if (opt.order_block < 1 || opt.order_block > 16)
    return fail(HLB_EINVAL, "order_block must be in 1..16 (got %d)", opt.order_block);
  if (opt.ladd_rho_local != 0 && opt.ladd_rho_local != 1)
    return fail(HLB_EINVAL, "ladd_rho_local must be 0 or 1 (got %d)", opt.ladd_rho_local);
  if (opt.ladd_rho_local && opt.adjoint)
    return fail(HLB_EINVAL, "the adjoint takes the Ladd rule with rho0 (ladd_rho_local must be 0)");
  if (!(opt.rho0 > 0.0) || !std::isfinite(opt.rho0)) return fail(HLB_EINVAL, "rho0 must be finite and > 0");
  if ((opt.adjoint != 0 && opt.adjoint != 1) || opt.max_device_bytes < 0 || opt.xcd_remap < -1 ||
      opt.xcd_remap > (1 << 20))
    return fail(HLB_EINVAL, "bad options");
  if (opt.adjoint && opt.storage != HLB_F64) return fail(HLB_EINVAL, "the adjoint needs FP64 storage");
  if (opt.scheme != HLB_SCHEME_PULL && opt.scheme != HLB_SCHEME_PUSH) return fail(HLB_EINVAL, "bad scheme %d", opt.scheme);
  if (opt.sites_per_thread < 0 || opt.sites_per_thread > 2)
    return fail(HLB_EINVAL, "sites_per_thread must be 0, 1 or 2 (got %d)", opt.sites_per_thread);
  if (opt.graph_steps < 0 || opt.graph_steps % 2 != 0 || opt.graph_steps > 4096)
    return fail(HLB_EINVAL, "graph_steps must be 0 or even in 2..4096 (got %d)", opt.graph_steps);
  if (opt.adjoint && opt.scheme != HLB_SCHEME_PULL) return fail(HLB_EINVAL, "the adjoint needs the pull scheme");
  int64_t n_ghost = 0;
  if (role) {
    if (opt.adjoint || opt.scheme != HLB_SCHEME_PULL)
      return fail(HLB_EINVAL, "a partition needs the pull scheme and no adjoint");
    for (int64_t x = 0; x < n; ++x) {
      if (role[x] > HLB_PART_GHOST) return fail(HLB_EINVAL, "site %lld: bad role %d", (long long)x, (int)role[x]);
      n_ghost += role[x] == HLB_PART_GHOST;
    }
    if (n_ghost == n) return fail(HLB_EINVAL, "a partition needs at least one owned site");
  }
  auto is_ghost = [&](int64_t x) { return role && role[x] == HLB_PART_GHOST; };
  for (int k = 0; k < n_iolets; ++k) {
    const hlb_iolet &I = iolets[k];
    if (I.kind != HLB_IOLET_VELOCITY && I.kind != HLB_IOLET_PRESSURE) return fail(HLB_EINVAL, "iolet %d: bad kind", k);
    if (I.role != HLB_ROLE_INLET && I.role != HLB_ROLE_OUTLET) return fail(HLB_EINVAL, "iolet %d: bad role", k);
    const double nn = std::sqrt(I.normal[0] * I.normal[0] + I.normal[1] * I.normal[1] + I.normal[2] * I.normal[2]);
    if (!(std::fabs(nn - 1.0) < 1e-6)) return fail(HLB_EINVAL, "iolet %d: normal is not a unit vector", k);
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(I.centre[a]) || !std::isfinite(I.vdir[a])) return fail(HLB_EINVAL, "iolet %d: non-finite", k);
    if (!std::isfinite(I.radius)) return fail(HLB_EINVAL, "iolet %d: non-finite radius", k);
  }

  // ---- validation of the tables (first offending site reported) ----
  int64_t bad_site = INT64_MAX;
  int bad_kind = 0;
#pragma omp parallel for schedule(static) reduction(min : bad_site)
  for (int64_t x = 0; x < n; ++x) {
    const int32_t *row = nbr + Q * x;
    bool ok = row[0] == x;
    bool wall = false;
    int roles = 0;
    for (int a = 0; a < 3 && ok; ++a) ok = coords[3 * x + a] >= 0 && coords[3 * x + a] < (1 << 20);
    if (is_ghost(x)) {
      if (!ok && x < bad_site) bad_site = x;
      continue;  // a ghost's links and type are not used
    }
    for (int i = 1; i < Q && ok; ++i) {
      const int32_t y = row[i];
      if (y >= 0) {
        ok = y < n && (is_ghost(y) || nbr[Q * (int64_t)y + OPP(i)] == x);
      } else if (y == HLB_LINK_WALL) {
        wall = true;
      } else {
        const int32_t k = -(y + 2);
        ok = k >= 0 && k < n_iolets;
        if (ok) roles |= iolets[k].role == HLB_ROLE_INLET ? 1 : 2;
      }
    }
    if (ok) {
      int want;
      if (roles == 3) want = -1;
      else if (roles == 1) want = wall ? HLB_SITE_INLET_WALL : HLB_SITE_INLET;
      else if (roles == 2) want = wall ? HLB_SITE_OUTLET_WALL : HLB_SITE_OUTLET;
      else want = wall ? HLB_SITE_WALL : HLB_SITE_BULK;
      ok = (int)type[x] == want;
    }
    if (!ok && x < bad_site) bad_site = x;
  }
  if (bad_site != INT64_MAX) {
    const int64_t x = bad_site;
    const int32_t *row = nbr + Q * x;
    (void)bad_kind;
    if (row[0] != x) return fail(HLB_EINVAL, "site %lld: nbr[x][0] must be x", (long long)x);
    for (int a = 0; a < 3; ++a)
      if (coords[3 * x + a] < 0 || coords[3 * x + a] >= (1 << 20))
        return fail(HLB_EINVAL, "site %lld: coordinate out of [0, 2^20)", (long long)x);
    for (int i = 1; i < Q; ++i) {
      const int32_t y = row[i];
      if (y >= n) return fail(HLB_EINVAL, "site %lld link %d: neighbour id %d out of range", (long long)x, i, y);
      if (is_ghost(x)) break;
      if (y >= 0 && !is_ghost(y) && nbr[Q * (int64_t)y + OPP(i)] != x)
        return fail(HLB_EINVAL, "site %lld link %d: neighbour table not symmetric", (long long)x, i);
      if (y < HLB_LINK_WALL && -(y + 2) >= n_iolets)
        return fail(HLB_EINVAL, "site %lld link %d: iolet id %d out of range", (long long)x, i, -(y + 2));
    }
    return fail(HLB_EINVAL, "site %lld: site type %d disagrees with its link codes", (long long)x, (int)type[x]);
  }

  hlb_ctx *c = new (std::nothrow) hlb_ctx();
  if (!c) return fail(HLB_ENOMEM, "host allocation");
  c->cfg.storage = opt.storage;
  c->cfg.tau = tau;
  c->cfg.rho0 = opt.rho0;
  c->cfg.xcd_chunk = opt.xcd_remap;
  c->cfg.porous = false;
  c->cfg.scheme = opt.scheme;
  c->cfg.sites_per_thread = opt.sites_per_thread > 0 ? opt.sites_per_thread : default_sites_per_thread(opt.storage);
  c->cfg.ladd_local = opt.ladd_rho_local != 0;
  c->graph_steps = opt.graph_steps;
  c->order = opt.order;
  c->max_bytes = opt.max_device_bytes;
  c->iolets.assign(iolets, iolets + n_iolets);
  c->tables.resize(n_iolets);
  for (int k = 0; k < n_iolets; ++k)
    c->tables[k] = {iolets[k].kind == HLB_IOLET_VELOCITY ? 0.0 : opt.rho0};

  // ---- grouping and space-filling-curve order within each group ----
  Layout &L = c->L;
  L.n_sites = n;
  std::vector<std::vector<KeyId>> grp(kGroups);
  {
    std::vector<int64_t> cnt(kGroups, 0);
    for (int64_t x = 0; x < n; ++x)
      if (!is_ghost(x)) cnt[group_of(type[x])]++;
    for (int g = 0; g < kGroups; ++g) grp[g].resize(cnt[g]);
    std::vector<int64_t> fill(kGroups, 0);
    for (int64_t x = 0; x < n; ++x) {
      if (is_ghost(x)) continue;
      const int g = group_of(type[x]);
      grp[g][fill[g]++] = KeyId(0, (int32_t)x);
    }
    KeyGeom kg;
    kg.b = opt.order_block;
    for (int64_t x = 0; x < n; ++x) {
      kg.nx = std::max<uint64_t>(kg.nx, (uint64_t)coords[3 * x] + 1);
      kg.ny = std::max<uint64_t>(kg.ny, (uint64_t)coords[3 * x + 1] + 1);
      kg.nz = std::max<uint64_t>(kg.nz, (uint64_t)coords[3 * x + 2] + 1);
    }
    for (int g = 0; g < kGroups; ++g) {
      auto &v = grp[g];
#pragma omp parallel for schedule(static)
      for (int64_t k = 0; k < (int64_t)v.size(); ++k) {
        const int32_t x = v[k].second;
        uint64_t key = sfc_key(opt.order, x, coords + 3 * (int64_t)x, kg);
        // a partition's edge sites lead the bulk+wall group (bit 63 is
        // unused by every order's key)
        if (g == 0 && role && role[x] != HLB_PART_EDGE) key |= uint64_t(1) << 63;
        v[k].first = key;
      }
      psort(v);
    }
    int64_t n_edge0 = 0;
    if (role)
      for (const KeyId &kv : grp[0]) n_edge0 += role[kv.second] == HLB_PART_EDGE;
    L.edge_blocks = (n_edge0 + kSegBlock - 1) / kSegBlock;
  }
  int64_t pos = 0;
  for (int g = 0; g < kGroups; ++g) {
    L.gbeg[g] = pos;
    L.gcnt[g] = (int64_t)grp[g].size();
    pos += L.gcnt[g];
    pos = (pos + kGroupAlign - 1) / kGroupAlign * kGroupAlign;
  }
  L.gbeg[kGroups] = pos;
  // ghost positions follow the groups, in caller order, from a tile of
  // their own: peers may write them while this partition's kernels write
  // the owned positions, so no cache line holds both
  if (n_ghost > 0) pos = (pos + kPopTile - 1) / kPopTile * kPopTile;
  L.ghost_begin = pos;
  L.n_ghost = n_ghost;
  pos += n_ghost;
  L.np = (std::max<int64_t>(pos, 1) + kPopTile - 1) / kPopTile * kPopTile;
  L.io_begin = L.gbeg[1];
  L.nio = L.np - L.io_begin;
  const int64_t np = L.np;
  if (opt.xcd_remap < 0) c->cfg.xcd_chunk = auto_xcd_chunk(opt.storage, np);
  c->order_host.assign(np, -1);
  std::vector<int32_t> inv(n);
  for (int g = 0; g < kGroups; ++g)
    for (int64_t k = 0; k < L.gcnt[g]; ++k) {
      const int32_t x = grp[g][k].second;
      c->order_host[L.gbeg[g] + k] = x;
      inv[x] = (int32_t)(L.gbeg[g] + k);
    }
  // ghosts: positions for the pull tables, no caller id (order -1), so that
  // no kernel updates them and macros, mass and state export skip them
  {
    int64_t k = 0;
    for (int64_t x = 0; x < n; ++x)
      if (is_ghost(x)) inv[x] = (int32_t)(L.ghost_begin + k++);
  }
  if (role) {
    c->role_host.assign(role, role + n);
    c->inv_host = inv;
  }
  grp.clear();
  grp.shrink_to_fit();

  // ---- pull tables: population i of position p comes from the site at x - c_i ----
  // Iolet groups: per-link table of source positions or link codes
  // (-1 wall, -(2+k) iolet k).
  std::vector<int32_t> pull_io((size_t)18 * L.nio, HLB_LINK_WALL);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < L.nio; ++q) {
    const int32_t x = c->order_host[L.io_begin + q];
    if (x < 0) continue;
    for (int i = 1; i < Q; ++i) {
      const int32_t y = nbr[Q * (int64_t)x + OPP(i)];
      pull_io[(size_t)(i - 1) * L.nio + q] = y >= 0 ? inv[y] : y;
    }
  }
  // Bulk+wall group: segmented source offsets (see kSegRow in hlb_internal.h).
  const int64_t n0 = L.gcnt[0];
  const int64_t nb0 = (n0 + kSegBlock - 1) / kSegBlock;
  auto offset_of = [&](int64_t p, int i) -> int32_t {
    const int32_t y = nbr[Q * (int64_t)c->order_host[p] + OPP(i)];
    return y >= 0 ? (int32_t)(inv[y] - p) : (int32_t)np;
  };
  std::vector<int32_t> segid(n0);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n0; ++p) {
    bool start = p == 0;
    for (int i = 1; i < Q && !start; ++i) start = offset_of(p, i) != offset_of(p - 1, i);
    segid[p] = start ? 1 : 0;
  }
  int64_t nseg = 0;
  for (int64_t p = 0; p < n0; ++p) {
    nseg += segid[p];
    segid[p] = (int32_t)(nseg - 1);
  }
  L.nseg = nseg;
  // one padding row after the last segment (read by a wavefront's scalar
  // row loads, never used)
  std::vector<int32_t> seg_off((size_t)kSegRow * (nseg + 1), 0);
  std::vector<int32_t> seg_base(std::max<int64_t>(nb0, 1), 0);
  std::vector<uint8_t> seg_delta((size_t)std::max<int64_t>(nb0 * kSegBlock, 1), 0);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n0; ++p) {
    if (p == 0 || segid[p] != segid[p - 1])
      for (int i = 1; i < Q; ++i) seg_off[(size_t)segid[p] * kSegRow + (i - 1)] = offset_of(p, i);
    if (p % kSegBlock == 0) seg_base[p / kSegBlock] = segid[p];
  }
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n0; ++p) seg_delta[p] = (uint8_t)(segid[p] - segid[(p / kSegBlock) * kSegBlock]);
  segid.clear();
  segid.shrink_to_fit();
  // the adjoint's transposed gather reads the pull tables; it only needs the
  // list of the sites with wall or iolet links (boundary terms)
  c->adj_on = opt.adjoint != 0;
  std::vector<int32_t> blist;
  if (c->adj_on)
    for (int64_t p = 0; p < np; ++p) {
      const int32_t x = c->order_host[p];
      if (x < 0) continue;
      bool any = false;
      for (int i = 1; i < Q && !any; ++i) any = nbr[Q * (int64_t)x + i] < 0;
      if (any) blist.push_back((int32_t)p);
    }
  // ---- Ladd coefficients 6 w_i rho0 (c_i . v_k) W_k(x - c_i/2) of velocity-iolet links ----
  std::vector<double> corr((size_t)18 * L.nio, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < L.nio; ++q) {
    const int32_t x = c->order_host[L.io_begin + q];
    if (x < 0) continue;
    for (int i = 1; i < Q; ++i) {
      const int32_t y = nbr[Q * (int64_t)x + OPP(i)];
      if (y > HLB_LINK_IOLET(0)) continue;
      const hlb_iolet &I = iolets[-(y + 2)];
      if (I.kind != HLB_IOLET_VELOCITY) continue;
      const double m[3] = {coords[3 * (int64_t)x] - 0.5 * CX[i], coords[3 * (int64_t)x + 1] - 0.5 * CY[i],
                           coords[3 * (int64_t)x + 2] - 0.5 * CZ[i]};
      double wgt = 1.0;
      if (I.radius > 0.0) {
        const double r[3] = {m[0] - I.centre[0], m[1] - I.centre[1], m[2] - I.centre[2]};
        const double along = r[0] * I.normal[0] + r[1] * I.normal[1] + r[2] * I.normal[2];
        const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] - along * along;
        wgt = std::max(0.0, 1.0 - d2 / (I.radius * I.radius));
      }
      const double *v = (I.vdir[0] == 0.0 && I.vdir[1] == 0.0 && I.vdir[2] == 0.0) ? I.normal : I.vdir;
      const double cv = CX[i] * v[0] + CY[i] * v[1] + CZ[i] * v[2];
      corr[(size_t)(i - 1) * L.nio + q] = 6.0 * W(i) * opt.rho0 * cv * wgt;
    }
  }

  // ---- device set-up (Sec. 3.2.1) ----
  auto bail = [&](hlb_status st) {
    std::string msg = g_err;
    free_all(c);
    delete c;
    g_err = msg;
    return st;
  };
  hipError_t he = hipGetDevice(&c->device);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(HLB_EDEVICE, "no HIP device: %s", hipGetErrorString(he));
  }
  // device address of the allocation-free reduction's partial sums, looked
  // up once per device here so that hlb_mass_balance_noalloc never has to
  if ((he = noalloc_setup(nullptr)) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(HLB_EDEVICE, "hipGetSymbolAddress of the reduction scratch: %s", hipGetErrorString(he));
  }
  const size_t fb = (size_t)Q * np * storage_bytes(opt.storage);
  const int64_t partial_len = 1 + 8192;
  const size_t need = 2 * fb + pull_io.size() * sizeof(int32_t) + seg_off.size() * sizeof(int32_t) +
                      seg_base.size() * sizeof(int32_t) + seg_delta.size() + np * sizeof(int32_t) +
                      corr.size() * sizeof(double) + partial_len * sizeof(double);
  if (c->max_bytes > 0 && (int64_t)need > c->max_bytes) {
    delete c;
    return fail(HLB_ENOMEM, "needs %zu device bytes, budget is %lld", need, (long long)opt.max_device_bytes);
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need > free_b) {
    delete c;
    return fail(HLB_ENOMEM, "needs %zu device bytes, %zu free", need, free_b);
  }
  if (hipStreamCreate(&c->own_stream) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(HLB_EDEVICE, "hipStreamCreate failed");
  }
  c->stream = c->own_stream;
  void *p = nullptr;
  hlb_status st;
  if ((st = dev_alloc(c, &c->d.f[0], fb))) return bail(st);
  if ((st = dev_alloc(c, &c->d.f[1], fb))) return bail(st);
  if ((st = dev_alloc(c, &p, std::max<size_t>(1, pull_io.size()) * sizeof(int32_t)))) return bail(st);
  c->d.nbr_io = static_cast<int32_t *>(p);
  if ((st = dev_alloc(c, &p, seg_off.size() * sizeof(int32_t)))) return bail(st);
  c->d.seg_off = static_cast<int32_t *>(p);
  if ((st = dev_alloc(c, &p, seg_base.size() * sizeof(int32_t)))) return bail(st);
  c->d.seg_base = static_cast<int32_t *>(p);
  if ((st = dev_alloc(c, &p, seg_delta.size()))) return bail(st);
  c->d.seg_delta = static_cast<uint8_t *>(p);
  c->table_bytes = (int64_t)(pull_io.size() * sizeof(int32_t) + seg_off.size() * sizeof(int32_t) +
                             seg_base.size() * sizeof(int32_t) + seg_delta.size());
  if ((st = dev_alloc(c, &p, np * sizeof(int32_t)))) return bail(st);
  c->d.order = static_cast<int32_t *>(p);
  if ((st = dev_alloc(c, &p, std::max<size_t>(1, corr.size()) * sizeof(double)))) return bail(st);
  c->d.corr = static_cast<double *>(p);
  if ((st = dev_alloc(c, &p, 4 * sizeof(double)))) return bail(st);
  c->d.acc = static_cast<double *>(p);
  if ((st = dev_alloc(c, &p, partial_len * sizeof(double)))) return bail(st);
  c->d.partial = static_cast<double *>(p);
  c->d.partial_len = partial_len;
  auto cp = [&](void *dst, const void *src, size_t bytes) -> hlb_status {
    hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(HLB_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    return HLB_OK;
  };
  if (!pull_io.empty() && (st = cp(c->d.nbr_io, pull_io.data(), pull_io.size() * sizeof(int32_t)))) return bail(st);
  if ((st = cp(c->d.seg_off, seg_off.data(), seg_off.size() * sizeof(int32_t)))) return bail(st);
  if ((st = cp(c->d.seg_base, seg_base.data(), seg_base.size() * sizeof(int32_t)))) return bail(st);
  if ((st = cp(c->d.seg_delta, seg_delta.data(), seg_delta.size()))) return bail(st);
  if ((st = cp(c->d.order, c->order_host.data(), np * sizeof(int32_t)))) return bail(st);
  if (!blist.empty()) {
    if ((st = dev_alloc(c, &p, blist.size() * sizeof(int32_t)))) return bail(st);
    c->adj.blist = static_cast<int32_t *>(p);
    c->adj.n_blist = (int64_t)blist.size();
    c->adj.n_blist_wall =
        (int64_t)(std::lower_bound(blist.begin(), blist.end(), (int32_t)L.io_begin) - blist.begin());
    if ((st = cp(c->adj.blist, blist.data(), blist.size() * sizeof(int32_t)))) return bail(st);
  }
  if (!corr.empty() && (st = cp(c->d.corr, corr.data(), corr.size() * sizeof(double)))) return bail(st);
  if ((st = upload_tables(c))) return bail(st);
  if ((st = hlb_init_equilibrium(c, nullptr, nullptr, 0))) return bail(st);
  *out = c;
  return HLB_OK;
}

hlb_status hlb_destroy(hlb_ctx *c) {
  if (!c) return HLB_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return HLB_OK;
}

hlb_status hlb_set_stream(hlb_ctx *c, void *s) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->stream = s ? static_cast<hipStream_t>(s) : c->own_stream;
  return HLB_OK;
}

hlb_status hlb_set_mid_stream(hlb_ctx *c, void *s) {
  if (hlb_status st = check_ctx(c)) return st;
  if (c->split_pending) return fail(HLB_ESTATE, "hlb_step_mid is pending");
  c->mid_stream = static_cast<hipStream_t>(s);
  return HLB_OK;
}

hlb_status hlb_set_iolet_table(hlb_ctx *c, int32_t k, const double *v, int64_t len) {
  if (hlb_status st = check_ctx(c)) return st;
  if (k < 0 || k >= (int32_t)c->iolets.size()) return fail(HLB_EINVAL, "iolet %d out of range", k);
  if (!v || len < 1 || len > (1ll << 31)) return fail(HLB_EINVAL, "table must have 1..2^31 values");
  for (int64_t s = 0; s < len; ++s)
    if (!std::isfinite(v[s])) return fail(HLB_EINVAL, "table value %lld not finite", (long long)s);
  if (c->iolets[k].kind == HLB_IOLET_PRESSURE)
    for (int64_t s = 0; s < len; ++s)
      if (!(v[s] > 0.0)) return fail(HLB_EINVAL, "ghost density must be > 0");
  if (hlb_status st = bind(c)) return st;
  c->tables[k].assign(v, v + len);
  if (k < (int32_t)c->tab_dev.size()) c->tab_dev[k] = 0;  // the host copy is now the newer one
  if (k < (int32_t)c->wk_on.size() && c->wk_on[k]) {  // a table replaces the Windkessel
    c->wk_on[k] = 0;
    c->n_wk--;
  }
  return upload_tables(c);
}

hlb_status hlb_set_windkessel(hlb_ctx *c, int32_t k, const hlb_windkessel *w) {
  if (hlb_status st = check_ctx(c)) return st;
  const int K = (int)c->iolets.size();
  if (k < 0 || k >= K) return fail(HLB_EINVAL, "iolet %d out of range", k);
  if (c->iolets[k].kind != HLB_IOLET_PRESSURE) return fail(HLB_EINVAL, "iolet %d is not a pressure iolet", k);
  if (!c->role_host.empty()) return fail(HLB_EINVAL, "Windkessel outlets are not supported on a partition");
  if (w) {
    const double v[5] = {w->rho_ref, w->R1, w->C, w->R2, w->X0};
    for (double x : v)
      if (!std::isfinite(x)) return fail(HLB_EINVAL, "Windkessel parameters must be finite");
    if (!(w->R1 >= 0.0 && w->C >= 0.0 && w->R2 >= 0.0)) return fail(HLB_EINVAL, "R1, C, R2 must be >= 0");
    if (w->C > 0.0 && w->R2 > 0.0 && w->R2 * w->C < 1.0)
      return fail(HLB_EINVAL, "R2 C must be >= 1 (one explicit step per lattice step)");
    if (!(w->rho_ref + w->X0 > 0.0)) return fail(HLB_EINVAL, "the initial density rho_ref + X0 must be > 0");
  }
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (!c->d.wk) {
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, (size_t)K * sizeof(WkParams))) return st;
    c->d.wk = static_cast<WkParams *>(p);
    if (hlb_status st = dev_alloc(c, &p, (size_t)2 * K * sizeof(double))) return st;
    c->d.wk_rho = static_cast<double *>(p);
    if (hlb_status st = dev_alloc(c, &p, (size_t)K * sizeof(double))) return st;
    c->d.io_flux = static_cast<double *>(p);
    std::vector<double> z((size_t)2 * K, 0.0);
    HIP_TRY(hipMemcpy(c->d.wk_rho, z.data(), 2 * K * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d.io_flux, z.data(), K * sizeof(double), hipMemcpyHostToDevice));
    c->wk_on.assign(K, 0);
  }
  const bool was = c->wk_on[k] != 0;
  if (w) {
    const WkParams P{w->rho_ref, w->R1, w->C, w->R2, w->X0, 0.0};
    const double rho[2] = {w->rho_ref + w->X0, w->rho_ref + w->X0};
    const double zero = 0.0;
    HIP_TRY(hipMemcpy(c->d.wk + k, &P, sizeof(P), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d.wk_rho + 2 * k, rho, sizeof(rho), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d.io_flux + k, &zero, sizeof(zero), hipMemcpyHostToDevice));
    c->wk_on[k] = 1;
    c->n_wk += was ? 0 : 1;
  } else {
    c->wk_on[k] = 0;
    c->n_wk -= was ? 1 : 0;
  }
  return upload_tables(c);
}

hlb_status hlb_windkessel_state(hlb_ctx *c, int32_t k, double *rho_next, double *X, double *Q_last) {
  if (hlb_status st = check_ctx(c)) return st;
  if (k < 0 || k >= (int32_t)c->iolets.size() || k >= (int32_t)c->wk_on.size() || !c->wk_on[k])
    return fail(HLB_EINVAL, "iolet %d is not a Windkessel outlet", k);
  if (hlb_status st = bind(c)) return st;
  WkParams P;
  double rho = 0.0;
  HIP_TRY(hipMemcpyAsync(&P, c->d.wk + k, sizeof(P), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&rho, c->d.wk_rho + 2 * k + (c->t & 1), sizeof(rho), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (rho_next) *rho_next = rho;
  if (X) *X = P.X;
  if (Q_last) *Q_last = P.Q;
  return HLB_OK;
}

hlb_status hlb_set_porosity(hlb_ctx *c, const double *phi) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  if (!phi) {
    c->cfg.porous = false;
    return HLB_OK;
  }
  const int64_t n = c->L.n_sites, np = c->L.np;
  for (int64_t x = 0; x < n; ++x)
    if (!(phi[x] >= 0.0 && phi[x] <= 1.0)) return fail(HLB_EINVAL, "phi[%lld] not in [0,1]", (long long)x);
  std::vector<double> h(np, 0.0);
  for (int64_t p = 0; p < np; ++p)
    if (c->order_host[p] >= 0) h[p] = phi[c->order_host[p]];
  if (!c->d.phi) {
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, np * sizeof(double))) return st;
    c->d.phi = static_cast<double *>(p);
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(c->d.phi, h.data(), np * sizeof(double), hipMemcpyHostToDevice));
  c->cfg.porous = true;
  return HLB_OK;
}

hlb_status hlb_set_porosity_device(hlb_ctx *c, const void *phi) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  if (!phi) {
    c->cfg.porous = false;
    return HLB_OK;
  }
  const double *v = static_cast<const double *>(phi);
  if (hlb_status st = check_device_values(c, v, c->L.n_sites, kCheckUnit, "a porosity value is not in [0,1]"))
    return st;
  if (!c->d.phi) {
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, c->L.np * sizeof(double))) return st;
    c->d.phi = static_cast<double *>(p);
  }
  HIP_TRY(launch_from_caller(v, c->d.order, c->L.np, c->d.phi, c->stream));
  c->cfg.porous = true;
  return HLB_OK;
}

hlb_status hlb_set_iolet_table_device(hlb_ctx *c, int32_t k, const void *values, int64_t len) {
  if (hlb_status st = check_ctx(c)) return st;
  if (k < 0 || k >= (int32_t)c->iolets.size()) return fail(HLB_EINVAL, "iolet %d out of range", k);
  if (!values || len < 1 || len > (1ll << 31)) return fail(HLB_EINVAL, "table must have 1..2^31 values");
  if (hlb_status st = bind(c)) return st;
  const double *v = static_cast<const double *>(values);
  const bool pressure = c->iolets[k].kind == HLB_IOLET_PRESSURE;
  if (hlb_status st = check_device_values(c, v, len, pressure ? kCheckPositive : kCheckFinite,
                                          pressure ? "a ghost density is not finite and > 0"
                                                   : "a table value is not finite"))
    return st;
  const bool wk = k < (int32_t)c->wk_on.size() && c->wk_on[k];
  if (!wk && len == (int64_t)c->tables[k].size() && k < (int32_t)c->tab_off.size()) {
    // same length: overwrite the iolet's run of the concatenated table in place
    HIP_TRY(hipMemcpyAsync(c->d.tables + c->tab_off[k], v, (size_t)len * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
    c->tab_dev[k] = 1;
    return HLB_OK;
  }
  // a new length (or a Windkessel to replace): the concatenation is rebuilt
  // from the host copies
  std::vector<double> h((size_t)len);
  HIP_TRY(hipMemcpyAsync(h.data(), v, (size_t)len * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->tables[k] = std::move(h);
  if (k < (int32_t)c->tab_dev.size()) c->tab_dev[k] = 0;
  if (wk) {
    c->wk_on[k] = 0;
    c->n_wk--;
  }
  return upload_tables(c);
}

hlb_status hlb_create(int64_t n, const int32_t *coords, const uint8_t *type, const int32_t *nbr, double tau,
                      const hlb_iolet *iolets, int32_t n_iolets, const hlb_options *opt, hlb_ctx **out) {
  return create_impl(n, coords, type, nbr, tau, iolets, n_iolets, opt, nullptr, out);
}

hlb_status hlb_create_part(int64_t n, const int32_t *coords, const uint8_t *type, const int32_t *nbr, double tau,
                           const hlb_iolet *iolets, int32_t n_iolets, const hlb_options *opt, const uint8_t *role,
                           hlb_ctx **out) {
  if (!role) return fail(HLB_EINVAL, "role is null");
  return create_impl(n, coords, type, nbr, tau, iolets, n_iolets, opt, role, out);
}

hlb_status hlb_halo_set(hlb_ctx *c, int64_t n_send, const int32_t *send_site, const int32_t *send_dir,
                        void *send_buf, int64_t n_recv, const int32_t *recv_site, const int32_t *recv_dir,
                        void *recv_buf) {
  if (hlb_status st = check_ctx(c)) return st;
  if (c->role_host.empty()) return fail(HLB_ESTATE, "not a partition (hlb_create_part)");
  if (n_send < 0 || n_recv < 0 || (n_send > 0 && (!send_site || !send_dir || !send_buf)) ||
      (n_recv > 0 && (!recv_site || !recv_dir || !recv_buf)))
    return fail(HLB_EINVAL, "bad halo lists or buffers");
  const int64_t n = c->L.n_sites;
  std::vector<int32_t> sp(n_send), sd(n_send), rp(n_recv), rd(n_recv);
  for (int64_t k = 0; k < n_send; ++k) {
    const int32_t x = send_site[k], i = send_dir[k];
    if (x < 0 || x >= n || c->role_host[x] != HLB_PART_EDGE || i < 0 || i >= Q)
      return fail(HLB_EINVAL, "send entry %lld: needs an edge site and a direction in [0, 19)", (long long)k);
    sp[k] = c->inv_host[x];
    sd[k] = i;
  }
  for (int64_t k = 0; k < n_recv; ++k) {
    const int32_t x = recv_site[k], i = recv_dir[k];
    if (x < 0 || x >= n || c->role_host[x] != HLB_PART_GHOST || i < 0 || i >= Q)
      return fail(HLB_EINVAL, "receive entry %lld: needs a ghost site and a direction in [0, 19)", (long long)k);
    rp[k] = c->inv_host[x];
    rd[k] = i;
  }
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  free_halo(c);
  const size_t eb = storage_bytes(c->cfg.storage);
  void *p = nullptr;
  auto alloc_cp = [&](void **dst, const void *src, size_t bytes) -> hlb_status {
    if (hlb_status st = dev_alloc(c, dst, std::max<size_t>(bytes, 16))) return st;
    c->halo.bytes += (int64_t)std::max<size_t>(bytes, 16);
    if (src && bytes > 0) {
      hipError_t e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) return fail(HLB_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    }
    return HLB_OK;
  };
  hlb_status st;
  if ((st = alloc_cp(&p, sp.data(), n_send * sizeof(int32_t)))) return st;
  c->halo.send_pos = static_cast<int32_t *>(p);
  if ((st = alloc_cp(&p, sd.data(), n_send * sizeof(int32_t)))) return st;
  c->halo.send_dir = static_cast<int32_t *>(p);
  if ((st = alloc_cp(&p, rp.data(), n_recv * sizeof(int32_t)))) return st;
  c->halo.recv_pos = static_cast<int32_t *>(p);
  if ((st = alloc_cp(&p, rd.data(), n_recv * sizeof(int32_t)))) return st;
  c->halo.recv_dir = static_cast<int32_t *>(p);
  (void)eb;
  c->halo.send_buf = send_buf;
  c->halo.recv_buf = recv_buf;
  c->halo.defined = true;
  c->halo.n_send = n_send;
  c->halo.n_recv = n_recv;
  return HLB_OK;
}

hlb_status hlb_halo_pack(hlb_ctx *c) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!c->halo.defined && c->peers.empty()) return fail(HLB_ESTATE, "no halo lists (hlb_halo_set / hlb_halo_add_peer)");
  if (c->split_pending) return fail(HLB_ESTATE, "a split step is in progress");
  if (hlb_status st = bind(c)) return st;
  if (c->halo.defined)
    HIP_TRY(launch_halo(c->cfg, c->d, c->cur, c->halo.send_pos, c->halo.send_dir, c->halo.n_send, c->halo.send_buf,
                        true, c->stream));
  // the current state into the peers' current buffers
  for (const auto &q : c->peers)
    HIP_TRY(launch_pack_to_peer(c->cfg.storage, c->d.f[c->cur], q.pos, q.dir, q.n, q.buf[c->cur], q.elem, c->stream));
  return HLB_OK;
}

hlb_status hlb_halo_ghost_slots(hlb_ctx *c, int64_t n, const int32_t *site, const int32_t *dir, int64_t *elem,
                                void **buf) {
  if (hlb_status st = check_ctx(c)) return st;
  if (c->role_host.empty()) return fail(HLB_ESTATE, "not a partition (hlb_create_part)");
  if (n < 0 || (n > 0 && (!site || !dir || !elem)) || !buf) return fail(HLB_EINVAL, "bad ghost list or outputs");
  const int64_t ns = c->L.n_sites;
  for (int64_t k = 0; k < n; ++k) {
    const int32_t x = site[k], i = dir[k];
    if (x < 0 || x >= ns || c->role_host[x] != HLB_PART_GHOST || i < 0 || i >= Q)
      return fail(HLB_EINVAL, "entry %lld: needs a ghost site and a direction in [0, 19)", (long long)k);
  }
  for (int64_t k = 0; k < n; ++k) {
    // element index of (position q, direction i) in the tiled buffers
    const int64_t q = c->inv_host[site[k]];
    elem[k] = (((q >> kPopTileShift) * Q + dir[k]) << kPopTileShift) + (q & (kPopTile - 1));
  }
  buf[0] = c->d.f[0];
  buf[1] = c->d.f[1];
  return HLB_OK;
}

hlb_status hlb_halo_add_peer(hlb_ctx *c, int64_t n, const int32_t *site, const int32_t *dir, void *peer_buf0,
                             void *peer_buf1, const int64_t *peer_elem) {
  if (hlb_status st = check_ctx(c)) return st;
  if (c->role_host.empty()) return fail(HLB_ESTATE, "not a partition (hlb_create_part)");
  if (c->split_pending) return fail(HLB_ESTATE, "a split step is in progress");
  if (n < 1 || !site || !dir || !peer_buf0 || !peer_buf1 || !peer_elem)
    return fail(HLB_EINVAL, "bad peer list or buffers");
  const int64_t ns = c->L.n_sites;
  std::vector<int32_t> sp(n), sd(n);
  for (int64_t k = 0; k < n; ++k) {
    const int32_t x = site[k], i = dir[k];
    if (x < 0 || x >= ns || c->role_host[x] != HLB_PART_EDGE || i < 0 || i >= Q)
      return fail(HLB_EINVAL, "entry %lld: needs an edge site and a direction in [0, 19)", (long long)k);
    if (peer_elem[k] < 0) return fail(HLB_EINVAL, "entry %lld: negative peer element", (long long)k);
    sp[k] = c->inv_host[x];
    sd[k] = i;
  }
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  hlb_ctx::Peer q;
  q.n = n;
  q.buf[0] = peer_buf0;
  q.buf[1] = peer_buf1;
  void *p = nullptr;
  auto put = [&](void **dst, const void *src, size_t bytes) -> hlb_status {
    if (hlb_status st = dev_alloc(c, dst, bytes)) return st;
    q.bytes += (int64_t)bytes;
    hipError_t e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(HLB_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    return HLB_OK;
  };
  hlb_status st = put(&p, sp.data(), n * sizeof(int32_t));
  q.pos = static_cast<int32_t *>(p);
  if (!st) {
    st = put(&p, sd.data(), n * sizeof(int32_t));
    q.dir = static_cast<int32_t *>(p);
  }
  if (!st) {
    st = put(&p, peer_elem, n * sizeof(int64_t));
    q.elem = static_cast<int64_t *>(p);
  }
  if (st) {
    if (q.pos) (void)hipFree(q.pos);
    if (q.dir) (void)hipFree(q.dir);
    if (q.elem) (void)hipFree(q.elem);
    c->dev_bytes -= q.bytes;
    return st;
  }
  c->peers.push_back(q);
  return HLB_OK;
}

hlb_status hlb_halo_clear_peers(hlb_ctx *c) {
  if (hlb_status st = check_ctx(c)) return st;
  if (c->split_pending) return fail(HLB_ESTATE, "a split step is in progress");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  free_peers(c);
  return HLB_OK;
}

hlb_status hlb_halo_unpack(hlb_ctx *c) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!c->halo.defined) return fail(HLB_ESTATE, "no halo lists (hlb_halo_set)");
  if (c->split_pending) return fail(HLB_ESTATE, "a split step is in progress");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(launch_halo(c->cfg, c->d, c->cur, c->halo.recv_pos, c->halo.recv_dir, c->halo.n_recv, c->halo.recv_buf,
                      false, c->stream));
  return HLB_OK;
}

hlb_status hlb_step_edge(hlb_ctx *c) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!c->halo.defined && c->peers.empty()) return fail(HLB_ESTATE, "no halo lists (hlb_halo_set / hlb_halo_add_peer)");
  if (c->split_pending) return fail(HLB_ESTATE, "hlb_step_mid must follow hlb_step_edge");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(launch_step(c->cfg, c->L, c->d, c->cur, c->t, c->stream, nullptr, nullptr, 1));
  // the edge sites' new post-collision values, from the buffer being
  // written: into the send buffer, or straight into the peers' buffers of
  // the same index (the one their next step pulls from)
  if (c->halo.defined)
    HIP_TRY(launch_halo(c->cfg, c->d, 1 - c->cur, c->halo.send_pos, c->halo.send_dir, c->halo.n_send,
                        c->halo.send_buf, true, c->stream));
  for (const auto &q : c->peers)
    HIP_TRY(launch_pack_to_peer(c->cfg.storage, c->d.f[1 - c->cur], q.pos, q.dir, q.n, q.buf[1 - c->cur], q.elem,
                                c->stream));
  c->split_pending = true;
  return HLB_OK;
}

hlb_status hlb_step_mid(hlb_ctx *c) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!c->split_pending) return fail(HLB_ESTATE, "hlb_step_edge must come first");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(launch_step(c->cfg, c->L, c->d, c->cur, c->t, c->mid_stream ? c->mid_stream : c->stream, nullptr, nullptr,
                      2));
  c->split_pending = false;
  c->cur = 1 - c->cur;
  c->direct = false;
  c->t += 1;
  return HLB_OK;
}

hlb_status hlb_set_objective(hlb_ctx *c, int32_t kind, const double *weights) {
  if (hlb_status st = check_ctx(c)) return st;
  if (kind == HLB_OBJ_WSS) {
    c->adj.objective = HLB_OBJ_WSS;
    return HLB_OK;
  }
  if (kind != HLB_OBJ_IOLET_FLUX) return fail(HLB_EINVAL, "unknown objective kind %d", (int)kind);
  const int64_t nio = (int64_t)c->iolets.size();
  if (nio > 0 && !weights) return fail(HLB_EINVAL, "the iolet-flux objective needs weights");
  for (int64_t k = 0; k < nio; ++k)
    if (!std::isfinite(weights[k])) return fail(HLB_EINVAL, "weights[%lld] is not finite", (long long)k);
  if (hlb_status st = bind(c)) return st;
  if (!c->adj.w) {
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, (size_t)std::max<int64_t>(nio, 1) * sizeof(double))) return st;
    c->adj.w = static_cast<double *>(p);
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (nio > 0) HIP_TRY(hipMemcpy(c->adj.w, weights, (size_t)nio * sizeof(double), hipMemcpyHostToDevice));
  c->adj.objective = HLB_OBJ_IOLET_FLUX;
  return HLB_OK;
}

hlb_status hlb_init_equilibrium(hlb_ctx *c, const double *rho, const double *u, int64_t t0) {
  if (hlb_status st = check_ctx(c)) return st;
  if (t0 < 0) return fail(HLB_EINVAL, "t0 < 0");
  if (hlb_status st = bind(c)) return st;
  const int64_t n = c->L.n_sites;
  const double *staging = nullptr;
  if (rho || u) {
    std::vector<double> h((size_t)n * 4);
    for (int64_t x = 0; x < n; ++x) {
      h[4 * x] = rho ? rho[x] : c->cfg.rho0;
      for (int a = 0; a < 3; ++a) h[4 * x + 1 + a] = u ? u[3 * x + a] : 0.0;
      if (!(h[4 * x] > 0.0) || !std::isfinite(h[4 * x + 1]) || !std::isfinite(h[4 * x + 2]) || !std::isfinite(h[4 * x + 3]))
        return fail(HLB_EINVAL, "bad initial rho/u at site %lld", (long long)x);
    }
    if (hlb_status st = ensure_staging(c, 4 * n)) return st;
    HIP_TRY(hipMemcpyAsync(c->d.io_scratch, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    staging = c->d.io_scratch;
    HIP_TRY(launch_init_eq(c->cfg, c->L, c->d, staging, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  } else {
    HIP_TRY(launch_init_eq(c->cfg, c->L, c->d, nullptr, c->stream));
  }
  c->cur = 0;
  c->direct = true;
  c->t = t0;
  return reset_balance(c);
}

// The buffer and mode the macros of the current state are read from: pull
// re-gathers the previous post-collision buffer (or reads the current
// pre-collision one right after init/set_state); push reads its current
// pre-collision buffer directly.
static void macro_source(const hlb_ctx *c, int *src, bool *direct) {
  if (c->cfg.scheme == HLB_SCHEME_PUSH) {
    *src = c->cur;
    *direct = true;
  } else {
    *src = 1 - c->cur;
    *direct = c->direct;
  }
}

namespace {

// Capture the graph of c->graph_steps steps that starts from buffer `cur`:
// step k reads the time as *t_dev + k, and a last node advances *t_dev, so
// that back-to-back replays continue the count.  Captured on a private
// stream (the context stream may be the null stream, which cannot capture).
hlb_status capture_steps(hlb_ctx *c, int cur) {
  if (!c->t_dev) {
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, sizeof(int64_t))) return st;
    c->t_dev = static_cast<int64_t *>(p);
  }
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  DevPtrs d = c->d;
  d.t_base = c->t_dev;
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < c->graph_steps && e == hipSuccess; ++k) {
    e = launch_step(c->cfg, c->L, d, (cur + k) & 1, k, c->cap_stream, nullptr, nullptr);
    if (e == hipSuccess && c->n_wk > 0) e = launch_windkessel(d, (int)c->iolets.size(), k, c->cap_stream);
  }
  if (e == hipSuccess) e = launch_add_time(c->t_dev, c->graph_steps, c->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&c->graph[cur], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->graph[cur] = nullptr;
    return fail(HLB_EDEVICE, "capturing the step graph: %s", hipGetErrorString(e));
  }
  return HLB_OK;
}

// reps replays of the step graph from the current time and buffer.
hlb_status replay_steps(hlb_ctx *c, int64_t reps) {
  if (!same_launch(c->graph_d, c->d) || !same_launch(c->graph_cfg, c->cfg) || c->graph_nwk != c->n_wk) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto &g : c->graph)
      if (g) {
        HIP_TRY(hipGraphExecDestroy(g));
        g = nullptr;
      }
    c->graph_d = c->d;
    c->graph_cfg = c->cfg;
    c->graph_nwk = c->n_wk;
  }
  if (!c->graph[c->cur])
    if (hlb_status st = capture_steps(c, c->cur)) return st;
  HIP_TRY(launch_set_time(c->t_dev, c->t, c->stream));
  for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(c->graph[c->cur], c->stream));
  // an even number of steps per graph: the state is back in buffer cur
  c->direct = false;
  c->t += reps * c->graph_steps;
  return HLB_OK;
}

}  // namespace

hlb_status hlb_step(hlb_ctx *c, int64_t n) {
  if (hlb_status st = check_ctx(c)) return st;
  if (n < 0) return fail(HLB_EINVAL, "n < 0");
  if (c->split_pending) return fail(HLB_ESTATE, "a split step is in progress (hlb_step_mid is due)");
  if (hlb_status st = bind(c)) return st;
  if (c->graph_steps > 0 && !c->timing && n >= c->graph_steps) {
    const int64_t reps = n / c->graph_steps;
    if (hlb_status st = replay_steps(c, reps)) return st;
    n -= reps * c->graph_steps;
  }
  for (int64_t s = 0; s < n; ++s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
      if (c->n_timed == c->pool.size()) {
        TimedStep ts;
        for (auto &e : ts.e) HIP_TRY(hipEventCreate(&e));
        c->pool.push_back(ts);
      }
      TimedStep &ts = c->pool[c->n_timed++];
      e0 = ts.e[0];
      e1 = ts.e[1];
    }
    HIP_TRY(launch_step(c->cfg, c->L, c->d, c->cur, c->t, c->stream, e0, e1));
    if (c->n_wk > 0) HIP_TRY(launch_windkessel(c->d, (int)c->iolets.size(), c->t, c->stream));
    c->cur = 1 - c->cur;
    c->direct = false;
    c->t += 1;
  }
  return HLB_OK;
}

hlb_status hlb_macros_device(hlb_ctx *c, void *rho, void *u, void *wss) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  if (!rho && !u && !wss) return HLB_OK;
  int src;
  bool direct;
  macro_source(c, &src, &direct);
  HIP_TRY(launch_macros(c->cfg, c->L, c->d, src, direct, c->t - 1, static_cast<double *>(rho),
                        static_cast<double *>(u), static_cast<double *>(wss), nullptr, c->stream));
  return HLB_OK;
}

hlb_status hlb_macros(hlb_ctx *c, double *rho, double *u, double *wss) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  if (!rho && !u && !wss) return HLB_OK;
  const int64_t n = c->L.n_sites;
  if (hlb_status st = ensure_staging(c, 5 * n)) return st;
  double *dr = c->d.io_scratch, *du = dr + n, *dw = du + 3 * n;
  int src;
  bool direct;
  macro_source(c, &src, &direct);
  HIP_TRY(launch_macros(c->cfg, c->L, c->d, src, direct, c->t - 1, rho ? dr : nullptr, u ? du : nullptr,
                        wss ? dw : nullptr, nullptr, c->stream));
  if (rho) HIP_TRY(hipMemcpyAsync(rho, dr, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (u) HIP_TRY(hipMemcpyAsync(u, du, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (wss) HIP_TRY(hipMemcpyAsync(wss, dw, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (rho)
    for (int64_t x = 0; x < n; ++x) {
      if (!c->role_host.empty() && c->role_host[x] == HLB_PART_GHOST) continue;  // unspecified
      if (!std::isfinite(rho[x])) return fail(HLB_ENUMERIC, "non-finite density at site %lld", (long long)x);
    }
  return HLB_OK;
}

hlb_status hlb_get_state(hlb_ctx *c, double *f) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!f) return fail(HLB_EINVAL, "f is null");
  if (hlb_status st = bind(c)) return st;
  if (hlb_status st = ensure_staging(c, Q * c->L.n_sites)) return st;
  int src;
  bool direct;
  macro_source(c, &src, &direct);
  HIP_TRY(launch_macros(c->cfg, c->L, c->d, src, direct, c->t - 1, nullptr, nullptr, nullptr, c->d.io_scratch,
                        c->stream));
  HIP_TRY(hipMemcpyAsync(f, c->d.io_scratch, (size_t)c->L.n_sites * Q * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HLB_OK;
}

hlb_status hlb_set_state(hlb_ctx *c, const double *f, int64_t t) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!f) return fail(HLB_EINVAL, "f is null");
  if (t < 0) return fail(HLB_EINVAL, "t < 0");
  const int64_t n = c->L.n_sites;
  for (int64_t k = 0; k < n * Q; ++k)
    if (!std::isfinite(f[k])) return fail(HLB_EINVAL, "f[%lld] not finite", (long long)k);
  if (hlb_status st = bind(c)) return st;
  if (hlb_status st = ensure_staging(c, Q * n)) return st;
  HIP_TRY(hipMemcpyAsync(c->d.io_scratch, f, (size_t)n * Q * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // buffer 1 := pre-collision f(t), buffer 0 := its collision; a pull step
  // reads the collided buffer, a push step the pre-collision one
  HIP_TRY(launch_set_state(c->cfg, c->L, c->d, 1, c->d.io_scratch, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->cur = c->cfg.scheme == HLB_SCHEME_PUSH ? 1 : 0;
  c->direct = true;
  c->t = t;
  return reset_balance(c);
}

hlb_status hlb_mass_balance_noalloc(hlb_ctx *c, void *out) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!out) return fail(HLB_EINVAL, "out is null");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(launch_mass_balance_noalloc(c->cfg, c->L, c->d, c->cur, mass_offset(c), c->m0, static_cast<double *>(out),
                                      c->stream));
  return HLB_OK;
}

hlb_status hlb_mass_balance(hlb_ctx *c, double *mass, double *residual) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  double s = 0.0, flux = 0.0;
  if (hlb_status st = compute_mass(c, &s)) return st;
  HIP_TRY(hipMemcpy(&flux, c->d.acc, sizeof(double), hipMemcpyDeviceToHost));
  const double M = mass_offset(c) + s;
  if (mass) *mass = M;
  if (residual) *residual = M - c->m0 - flux;
  if (!std::isfinite(M)) return fail(HLB_ENUMERIC, "total mass is not finite");
  return HLB_OK;
}

hlb_status hlb_time(const hlb_ctx *c, int64_t *t) {
  if (!c || !t) return fail(HLB_EINVAL, "null argument");
  *t = c->t;
  return HLB_OK;
}

hlb_status hlb_info(const hlb_ctx *c, hlb_info_t *info) {
  if (!c || !info) return fail(HLB_EINVAL, "null argument");
  std::memset(info, 0, sizeof(*info));
  info->n_sites = c->L.n_sites;
  info->n_padded = c->L.np;
  for (int g = 0; g < kGroups; ++g) info->group_sites[g] = c->L.gcnt[g];
  info->group_sites[kGroups] = c->L.n_ghost;
  info->storage = c->cfg.storage;
  info->order = c->order;
  // 19 loads + 19 stores of the populations, plus the pull tables (read once
  // per step), per site update
  info->table_bytes_per_site = (double)c->table_bytes / (double)c->L.n_sites;
  info->bytes_per_lup = 38.0 * (double)storage_bytes(c->cfg.storage) + info->table_bytes_per_site;
  info->n_segments = c->L.nseg;
  info->n_iolets = (int64_t)c->iolets.size();
  info->adjoint = c->adj_on ? 1 : 0;
  info->porous = c->cfg.porous ? 1 : 0;
  info->scheme = c->cfg.scheme;
  info->sites_per_thread = c->cfg.sites_per_thread;
  info->graph_steps = c->graph_steps;
  info->xcd_remap = c->cfg.xcd_chunk;
  info->device_bytes = c->dev_bytes;
  return HLB_OK;
}

hlb_status hlb_set_timing(hlb_ctx *c, int32_t enable) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  c->n_timed = 0;
  c->steps_timed = 0;
  c->sum_kernel = c->sum_step = 0.0;
  c->n_adj_timed = 0;
  c->adj_steps_timed = 0;
  c->sum_adj = 0.0;
  return HLB_OK;
}

hlb_status hlb_stats(hlb_ctx *c, hlb_stats_t *s) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!s) return fail(HLB_EINVAL, "null stats");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->n_timed > 0) {
    for (size_t k = 0; k < c->n_timed; ++k) {
      float a = 0;
      HIP_TRY(hipEventElapsedTime(&a, c->pool[k].e[0], c->pool[k].e[1]));
      c->sum_kernel += a;
    }
    float whole = 0;
    HIP_TRY(hipEventElapsedTime(&whole, c->pool[0].e[0], c->pool[c->n_timed - 1].e[1]));
    c->sum_step += whole;
    c->steps_timed += (int64_t)c->n_timed;
    c->n_timed = 0;
  }
  for (size_t k = 0; k < c->n_adj_timed; ++k) {
    float a = 0;
    HIP_TRY(hipEventElapsedTime(&a, c->adj_pool[k].e[0], c->adj_pool[k].e[1]));
    c->sum_adj += a;
  }
  c->adj_steps_timed += (int64_t)c->n_adj_timed;
  c->n_adj_timed = 0;
  s->steps = c->steps_timed;
  const double k = c->steps_timed > 0 ? (double)c->steps_timed : 1.0;
  s->kernel_ms = c->sum_kernel / k;
  s->step_ms = c->sum_step / k;
  s->adj_steps = c->adj_steps_timed;
  s->adj_ms = c->adj_steps_timed > 0 ? c->sum_adj / (double)c->adj_steps_timed : 0.0;
  // eq. (9) over the mean stream time per step; algorithmic bytes of a step
  // (hlb_info_t.bytes_per_lup per site) over the mean step-kernel duration
  const double n_upd = (double)(c->L.n_sites - c->L.n_ghost);
  const double bpl = 38.0 * (double)storage_bytes(c->cfg.storage) + (double)c->table_bytes / (double)c->L.n_sites;
  s->mlups = s->step_ms > 0.0 ? n_upd / (s->step_ms * 1e-3) / 1e6 : 0.0;
  s->alg_gbs = s->kernel_ms > 0.0 ? bpl * n_upd / (s->kernel_ms * 1e-3) / 1e9 : 0.0;
  return HLB_OK;
}

hlb_status hlb_snapshot_alloc(hlb_ctx *c, int32_t n_slots) {
  if (hlb_status st = check_ctx(c)) return st;
  if (n_slots < 0 || n_slots > 4096) return fail(HLB_EINVAL, "n_slots out of range");
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto &s : c->snaps) {
    if (s.f[0]) { (void)hipFree(s.f[0]); c->dev_bytes -= (int64_t)buf_bytes(c); }
    if (s.f[1]) { (void)hipFree(s.f[1]); c->dev_bytes -= (int64_t)buf_bytes(c); }
    if (s.acc) { (void)hipFree(s.acc); c->dev_bytes -= 4 * sizeof(double); }
  }
  c->snaps.assign(n_slots, hlb_ctx::Snap());
  for (auto &s : c->snaps) {
    if (hlb_status st = dev_alloc(c, &s.f[0], buf_bytes(c))) return st;
    if (hlb_status st = dev_alloc(c, &s.f[1], buf_bytes(c))) return st;
    void *p = nullptr;
    if (hlb_status st = dev_alloc(c, &p, 4 * sizeof(double))) return st;
    s.acc = static_cast<double *>(p);
  }
  return HLB_OK;
}

hlb_status hlb_snapshot_save(hlb_ctx *c, int32_t slot) {
  if (hlb_status st = check_ctx(c)) return st;
  if (slot < 0 || slot >= (int32_t)c->snaps.size()) return fail(HLB_EINVAL, "slot %d out of range", slot);
  if (hlb_status st = bind(c)) return st;
  auto &s = c->snaps[slot];
  HIP_TRY(hipMemcpyAsync(s.f[0], c->d.f[0], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(s.f[1], c->d.f[1], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(s.acc, c->d.acc, 4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  s.t = c->t; s.t0 = c->t0; s.m0 = c->m0; s.cur = c->cur; s.direct = c->direct; s.valid = true;
  return HLB_OK;
}

hlb_status hlb_snapshot_restore(hlb_ctx *c, int32_t slot) {
  if (hlb_status st = check_ctx(c)) return st;
  if (slot < 0 || slot >= (int32_t)c->snaps.size()) return fail(HLB_EINVAL, "slot %d out of range", slot);
  auto &s = c->snaps[slot];
  if (!s.valid) return fail(HLB_ESTATE, "slot %d holds no snapshot", slot);
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipMemcpyAsync(c->d.f[0], s.f[0], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d.f[1], s.f[1], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d.acc, s.acc, 4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->t = s.t; c->t0 = s.t0; c->m0 = s.m0; c->cur = s.cur; c->direct = s.direct;
  return HLB_OK;
}

namespace {
struct StateHeader {
  char magic[8];
  int64_t n_sites, np, t, t0;
  int32_t storage, cur, direct, scheme;
  double m0;
  double acc[4];
};
}  // namespace

hlb_status hlb_state_bytes(const hlb_ctx *c, int64_t *bytes) {
  if (!c || !bytes) return fail(HLB_EINVAL, "null argument");
  *bytes = (int64_t)(sizeof(StateHeader) + 2 * buf_bytes(c));
  return HLB_OK;
}

hlb_status hlb_state_save(hlb_ctx *c, void *buf) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!buf) return fail(HLB_EINVAL, "null buffer");
  if (hlb_status st = bind(c)) return st;
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "HLBSTAT2", 8);
  h.n_sites = c->L.n_sites; h.np = c->L.np; h.t = c->t; h.t0 = c->t0;
  h.storage = c->cfg.storage; h.cur = c->cur; h.direct = c->direct ? 1 : 0; h.m0 = c->m0;
  h.scheme = c->cfg.scheme;
  HIP_TRY(hipMemcpyAsync(h.acc, c->d.acc, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  char *b = static_cast<char *>(buf);
  HIP_TRY(hipMemcpyAsync(b + sizeof(h), c->d.f[0], buf_bytes(c), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(b + sizeof(h) + buf_bytes(c), c->d.f[1], buf_bytes(c), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(b, &h, sizeof(h));
  return HLB_OK;
}

hlb_status hlb_state_load(hlb_ctx *c, const void *buf) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!buf) return fail(HLB_EINVAL, "null buffer");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "HLBSTAT2", 8) != 0 || h.n_sites != c->L.n_sites || h.np != c->L.np ||
      h.storage != c->cfg.storage || h.scheme != c->cfg.scheme)
    return fail(HLB_EINVAL, "state buffer does not match this context");
  if (hlb_status st = bind(c)) return st;
  const char *b = static_cast<const char *>(buf);
  HIP_TRY(hipMemcpyAsync(c->d.f[0], b + sizeof(h), buf_bytes(c), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d.f[1], b + sizeof(h) + buf_bytes(c), buf_bytes(c), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d.acc, h.acc, 4 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->t = h.t; c->t0 = h.t0; c->m0 = h.m0; c->cur = h.cur; c->direct = h.direct != 0;
  return HLB_OK;
}

hlb_status hlb_sync(hlb_ctx *c) {
  if (hlb_status st = check_ctx(c)) return st;
  if (hlb_status st = bind(c)) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HLB_OK;
}

}  // extern "C"

namespace {

// C(n, k), saturating at 2^62.
int64_t binom_sat(int64_t n, int64_t k) {
  if (k < 0 || k > n) return 0;
  if (k > n - k) k = n - k;
  // v = C(n - k + i, i) after step i: exact in integers, saturated at 2^62
  __int128 v = 1;
  for (int64_t i = 1; i <= k; ++i) {
    v = v * (n - k + i) / i;
    if (v > ((__int128)1 << 62)) return (int64_t)1 << 62;
  }
  return (int64_t)v;
}

// Forward steps of the cheapest reversal of l steps with S checkpoint slots,
// the one holding the start state included (Griewank & Walther, binomial
// checkpointing): with r the least integer with C(S + r, S) >= l, it is
// r l - C(S + r, r - 1); l (l - 1) / 2 with the start state alone.
int64_t revolve_cost(int64_t l, int64_t S) {
  if (l <= 1) return 0;
  if (S <= 1) return l * (l - 1) / 2;
  int64_t r = 0;
  while (binom_sat(S + r, S) < l) ++r;
  return r * l - binom_sat(S + r, r - 1);
}

// Where to place the next checkpoint when l > 1 steps remain with S slots
// (S >= 2): m steps ahead, m in [1, l - 1] minimising
//   m + revolve_cost(l - m, S - 1) + revolve_cost(m, S)
// -- reach the checkpoint, reverse the part after it with one slot less,
// then the part before it with the slot freed again.  The sum is convex in
// m (each term is piecewise linear with growing slopes), so a bisection on
// its forward difference finds the minimum, and the recursion meets
// revolve_cost(l, S) exactly.
int64_t revolve_split(int64_t l, int64_t S) {
  auto cost = [&](int64_t m) { return m + revolve_cost(l - m, S - 1) + revolve_cost(m, S); };
  int64_t lo = 1, hi = l - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (cost(mid + 1) >= cost(mid)) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Forward steps the reverse sweep of Revolve takes from a to b with cfree
// free slots (a dry run of its recursion).
int64_t revolve_forward_steps(int64_t a, int64_t b, int64_t cfree) {
  int64_t fwd = 0;
  while (b - a > 1 && cfree > 0) {
    const int64_t m = a + revolve_split(b - a, cfree + 1);
    fwd += m - a + revolve_forward_steps(m, b, cfree - 1);
    b = m;
  }
  return fwd + (b - a) * (b - a - 1) / 2;  // each step recomputed from a
}

// Reverse sweep with binomial checkpointing (Griewank & Walther's schedule,
// written as a recursion): the state at time a is in slot `slot_a`, `cfree`
// more slots are free; adjoint steps b, b-1, ..., a+1 are run, each with
// the forward state of the preceding time restored or recomputed.  While
// slots are free, a checkpoint is placed revolve_split() steps ahead and
// the part after it is reversed first; with none free, each step is
// recomputed from a.  The forward steps total revolve_cost(n, n_snap).
struct Revolve {
  hlb_ctx *c;
  int64_t t0, n, w0, w1, n_snap;
  std::vector<int64_t> slot_t;
  int64_t fwd = 0;
  // The current state may live in a checkpoint slot instead of the
  // context's own buffer: a restore only points at the slot, the next forward
  // step pulls from it into a context buffer (or the adjoint step reads it
  // there), and a checkpoint's forward run writes its last step straight into
  // the slot.  No slot is written while it is read, so restores and
  // checkpoints cost no copy.
  const void *in_slot = nullptr;

  DevPtrs reading_slot() const {
    DevPtrs d = c->d;
    if (in_slot) d.f[c->cur] = const_cast<void *>(in_slot);
    return d;
  }
  // k forward steps; with `last_dst`, the last one writes into that slot.
  hlb_status advance(int64_t k, void *last_dst = nullptr) {
    for (int64_t s = 0; s < k; ++s) {
      DevPtrs d = reading_slot();
      void *dst = (last_dst && s == k - 1) ? last_dst : nullptr;
      if (dst) d.f[1 - c->cur] = dst;
      HIP_TRY(launch_step(c->cfg, c->L, d, c->cur, c->t, c->stream, nullptr, nullptr));
      if (c->n_wk > 0) HIP_TRY(launch_windkessel(c->d, (int)c->iolets.size(), c->t, c->stream));
      in_slot = dst;
      c->cur = 1 - c->cur;
      c->t += 1;
    }
    fwd += k;
    return HLB_OK;
  }
  // the Windkessel outlets' state to (or from) checkpoint slot `slot`
  hlb_status wk_state(int64_t slot, bool to_slot) {
    if (c->n_wk <= 0) return HLB_OK;
    const size_t nio = c->iolets.size(), pb = nio * sizeof(WkParams), rb = 2 * nio * sizeof(double);
    char *base = static_cast<char *>(c->adj_wk_slots) + (size_t)slot * (pb + rb);
    if (to_slot) {
      HIP_TRY(hipMemcpyAsync(base, c->d.wk, pb, hipMemcpyDeviceToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(base + pb, c->d.wk_rho, rb, hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIP_TRY(hipMemcpyAsync(c->d.wk, base, pb, hipMemcpyDeviceToDevice, c->stream));
      HIP_TRY(hipMemcpyAsync(c->d.wk_rho, base + pb, rb, hipMemcpyDeviceToDevice, c->stream));
    }
    return HLB_OK;
  }
  hlb_status save(int64_t slot) {
    const void *src = in_slot ? in_slot : c->d.f[c->cur];
    if (src != c->adj_slots[slot])
      HIP_TRY(hipMemcpyAsync(c->adj_slots[slot], src, buf_bytes(c), hipMemcpyDeviceToDevice, c->stream));
    slot_t[slot] = c->t;
    return wk_state(slot, true);
  }
  hlb_status restore(int64_t slot) {
    in_slot = c->adj_slots[slot];
    c->cur = 0;
    c->t = slot_t[slot];
    c->direct = false;
    return wk_state(slot, false);
  }
  hlb_status adjoint_step(int64_t t) {  // needs the state of time t-1
    const int in_window = (t > w0 && t <= w1) ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
      if (c->n_adj_timed == c->adj_pool.size()) {
        TimedStep ts;
        for (auto &e : ts.e) HIP_TRY(hipEventCreate(&e));
        c->adj_pool.push_back(ts);
      }
      TimedStep &ts = c->adj_pool[c->n_adj_timed++];
      e0 = ts.e[0];
      e1 = ts.e[1];
      HIP_TRY(hipEventRecord(e0, c->stream));
    }
    HIP_TRY(launch_adjoint_step(c->cfg, c->L, reading_slot(), c->cur, t, c->adj, in_window, n, t - 1 - t0,
                                c->stream));
    if (e1) HIP_TRY(hipEventRecord(e1, c->stream));
    return HLB_OK;
  }
  hlb_status reverse(int64_t a, int64_t b, int64_t slot_a, int64_t cfree) {
    while (b - a > 1 && cfree > 0) {
      const int64_t m = a + revolve_split(b - a, cfree + 1);
      const int64_t slot_m = n_snap - cfree;
      if (hlb_status st = restore(slot_a)) return st;
      if (hlb_status st = advance(m - a, c->adj_slots[slot_m])) return st;  // m - a >= 1
      slot_t[slot_m] = c->t;
      if (hlb_status st = wk_state(slot_m, true)) return st;
      if (hlb_status st = reverse(m, b, slot_m, cfree - 1)) return st;
      b = m;
    }
    for (int64_t t = b; t > a; --t) {  // no free slot left (or one step): recompute from a
      if (hlb_status st = restore(slot_a)) return st;
      if (hlb_status st = advance(t - 1 - a)) return st;
      if (hlb_status st = adjoint_step(t)) return st;
    }
    return HLB_OK;
  }
};

}  // namespace

extern "C" hlb_status hlb_revolve_forward_steps(int64_t n, int32_t n_snap, int64_t *steps) {
  if (n < 1 || n_snap < 1 || n_snap > 4096 || !steps) return fail(HLB_EINVAL, "need n >= 1, 1 <= n_snap <= 4096, steps");
  *steps = revolve_forward_steps(0, n, n_snap - 1);
  return HLB_OK;
}

namespace {

// The forward and reverse sweeps of hlb_adjoint_run, asynchronous on the
// context stream.  The objective, the table-value derivatives and the
// porosity derivatives (per position) are left in c->adj; the caller's
// state, time and flux bookkeeping are put back.
hlb_status adjoint_sweep(hlb_ctx *c, int64_t n, int64_t obj_t0, int64_t obj_t1, int32_t n_snap,
                         int64_t *forward_steps) {
  if (n < 1 || n_snap < 1 || n_snap > 4096) return fail(HLB_EINVAL, "need n >= 1, 1 <= n_snap <= 4096");
  if (c->cfg.storage != HLB_F64 || !c->adj_on || c->cfg.scheme != HLB_SCHEME_PULL || c->cfg.ladd_local)
    return fail(HLB_ESTATE, "the adjoint needs FP64 storage and opt.adjoint = 1 at creation");
  if (hlb_status st = bind(c)) return st;
  const int64_t np = c->L.np, nio = (int64_t)c->iolets.size();
  void *p = nullptr;
  if (!c->adj.mu) {
    if (hlb_status st = dev_alloc(c, &p, (size_t)Q * np * sizeof(double))) return st;
    c->adj.mu = static_cast<double *>(p);
    if (hlb_status st = dev_alloc(c, &p, (size_t)Q * np * sizeof(double))) return st;
    c->adj.nu = static_cast<double *>(p);
    if (hlb_status st = dev_alloc(c, &p, (size_t)np * sizeof(double))) return st;
    c->adj.dphi = static_cast<double *>(p);
    // [0] the objective; [1, 5) the caller's flux accumulators while the sweep runs
    if (hlb_status st = dev_alloc(c, &p, kAdjJLen * sizeof(double))) return st;
    c->adj.J = static_cast<double *>(p);
    if (hlb_status st = dev_alloc(c, &p, (size_t)std::max<int64_t>(1, nio) * sizeof(double))) return st;
    c->adj.wq = static_cast<double *>(p);
    if (hlb_status st = dev_alloc(c, &p, (size_t)std::max<int64_t>(1, nio) * sizeof(double))) return st;
    c->adj.lamX = static_cast<double *>(p);
  }
  c->adj.n_io = (int32_t)nio;
  // the Windkessel outlets' state per checkpoint slot
  if (c->n_wk > 0 && c->adj_wk_nslots < (int64_t)n_snap + 1) {
    if (c->adj_wk_slots) {
      (void)hipFree(c->adj_wk_slots);
      c->dev_bytes -= c->adj_wk_nslots * (int64_t)(nio * (sizeof(WkParams) + 2 * sizeof(double)));
      c->adj_wk_slots = nullptr;
      c->adj_wk_nslots = 0;
    }
    if (hlb_status st = dev_alloc(c, &p, (size_t)(n_snap + 1) * nio * (sizeof(WkParams) + 2 * sizeof(double))))
      return st;
    c->adj_wk_slots = p;
    c->adj_wk_nslots = (int64_t)n_snap + 1;
  }
  if (c->adj_dA_len < std::max<int64_t>(1, nio * n)) {
    if (c->adj.dA) {
      (void)hipFree(c->adj.dA);
      c->dev_bytes -= c->adj_dA_len * (int64_t)sizeof(double);
      c->adj.dA = nullptr;
      c->adj_dA_len = 0;
    }
    if (hlb_status st = dev_alloc(c, &p, (size_t)std::max<int64_t>(1, nio * n) * sizeof(double))) return st;
    c->adj.dA = static_cast<double *>(p);
    c->adj_dA_len = std::max<int64_t>(1, nio * n);
  }
  // checkpoint slots, plus one for the caller's other population buffer
  while ((int64_t)c->adj_slots.size() < (int64_t)n_snap + 1) {
    if (hlb_status st = dev_alloc(c, &p, buf_bytes(c))) return st;
    c->adj_slots.push_back(p);
  }
  // keep the caller's state: both buffers, time, flags, flux accumulator
  const int cur0 = c->cur;
  const bool direct0 = c->direct;
  const int64_t t_start = c->t;
  HIP_TRY(hipMemcpyAsync(c->adj.J + 1, c->d.acc, 4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->adj_slots[n_snap], c->d.f[1 - cur0], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(launch_zero(c->adj.mu, (int64_t)Q * np, c->stream));
  HIP_TRY(launch_zero(c->adj.dphi, np, c->stream));
  HIP_TRY(launch_zero(c->adj.J + 8, kAdjJSlots, c->stream));
  HIP_TRY(launch_zero(c->adj.dA, std::max<int64_t>(1, nio * n), c->stream));
  HIP_TRY(launch_zero(c->adj.lamX, std::max<int64_t>(1, nio), c->stream));
  Revolve R;
  R.c = c;
  R.t0 = t_start;
  R.n = n;
  R.w0 = obj_t0;
  R.w1 = obj_t1;
  R.n_snap = n_snap;
  R.slot_t.assign(n_snap, 0);
  hlb_status st = R.save(0);
  if (!st) st = R.reverse(t_start, t_start + n, 0, n_snap - 1);
  if (!st) {
    hipError_t e = launch_adjoint_objective(c->adj.J, c->stream);
    if (e != hipSuccess) st = fail(HLB_EDEVICE, "objective sum: %s", hipGetErrorString(e));
  }
  // put the caller's state back
  if (!st) {
    hipError_t e = hipMemcpyAsync(c->d.f[cur0], c->adj_slots[0], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->d.f[1 - cur0], c->adj_slots[n_snap], buf_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->d.acc, c->adj.J + 1, 4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) st = fail(HLB_EDEVICE, "restoring the state: %s", hipGetErrorString(e));
    if (!st) st = R.wk_state(0, false);
  }
  c->cur = cur0;
  c->direct = direct0;
  c->t = t_start;
  if (!st && forward_steps) *forward_steps = R.fwd;
  return st;
}

}  // namespace

extern "C" hlb_status hlb_adjoint_run(hlb_ctx *c, int64_t n, int64_t obj_t0, int64_t obj_t1, int32_t n_snap,
                                      double *J, double *dJ_dA, double *dJ_dphi, int64_t *forward_steps) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!J) return fail(HLB_EINVAL, "J is null");
  int64_t fwd = 0;
  if (hlb_status st = adjoint_sweep(c, n, obj_t0, obj_t1, n_snap, &fwd)) return st;
  const int64_t np = c->L.np, nio = (int64_t)c->iolets.size();
  HIP_TRY(hipMemcpyAsync(J, c->adj.J, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (dJ_dA && nio > 0)
    HIP_TRY(hipMemcpyAsync(dJ_dA, c->adj.dA, (size_t)nio * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  std::vector<double> dphi_pos;
  if (dJ_dphi) {
    dphi_pos.resize(np);
    HIP_TRY(hipMemcpyAsync(dphi_pos.data(), c->adj.dphi, np * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (dJ_dphi)
    for (int64_t q = 0; q < np; ++q)
      if (c->order_host[q] >= 0) dJ_dphi[c->order_host[q]] = dphi_pos[q];
  if (forward_steps) *forward_steps = fwd;
  if (!std::isfinite(*J)) return fail(HLB_ENUMERIC, "objective is not finite");
  return HLB_OK;
}

extern "C" hlb_status hlb_adjoint_run_device(hlb_ctx *c, int64_t n, int64_t obj_t0, int64_t obj_t1, int32_t n_snap,
                                             void *J, void *dJ_dA, void *dJ_dphi, int64_t *forward_steps) {
  if (hlb_status st = check_ctx(c)) return st;
  if (!J) return fail(HLB_EINVAL, "J is null");
  int64_t fwd = 0;
  if (hlb_status st = adjoint_sweep(c, n, obj_t0, obj_t1, n_snap, &fwd)) return st;
  const int64_t nio = (int64_t)c->iolets.size();
  HIP_TRY(hipMemcpyAsync(J, c->adj.J, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (dJ_dA && nio > 0)
    HIP_TRY(hipMemcpyAsync(dJ_dA, c->adj.dA, (size_t)nio * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (dJ_dphi) HIP_TRY(launch_to_caller(c->adj.dphi, c->d.order, c->L.np, static_cast<double *>(dJ_dphi), c->stream));
  if (forward_steps) *forward_steps = fwd;
  return HLB_OK;
}
