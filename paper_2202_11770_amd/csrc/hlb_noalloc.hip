// The FP64 mass balance without any allocation (hlb_mass_balance_noalloc):
// the partial sums of the reduction live in a file-scope device array of
// fixed size instead of the context's reduction buffer, and the result is
// written to the caller's device memory, so the call neither allocates nor
// waits and can sit in a captured graph or a loop that must not allocate.
#include <mutex>

#include "hlb_device.h"
#include "hlb_noalloc.h"

namespace {
constexpr int64_t kScratchDoubles = 1 + hlb::kNoAllocPartials;
}

// Partial sums of the reduction, one slot per workgroup (slot 0 unused), on
// every GPU the library runs on.  Host code must not pass this name to a
// kernel: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress (noalloc_setup).
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace hlb {
namespace {

using namespace dev;

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Same arithmetic and summation order as the context's own reduction
// (k_mass_partial / k_mass_final): the results are bit-identical.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mass_partial_na(const T *__restrict__ A, const int32_t *__restrict__ order,
                                                            int64_t np, double *partial) {
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

// out[0] = offset + sum of the partials (the total mass), out[1] = out[0] -
// m0 - acc[0] (the balance residual).
__global__ __launch_bounds__(kBlock) void k_mass_balance_na(const double *partial, int64_t nparts, double offset,
                                                            double m0, const double *acc, double *out) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nparts; k += kBlock) s += partial[1 + k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) b += red[w];
    const double M = offset + b;
    out[0] = M;
    out[1] = M - m0 - acc[0];
  }
}

template <typename T>
hipError_t mass_na(const Layout &L, const DevPtrs &d, int src, double offset, double m0, double *scr, double *out,
                   hipStream_t s) {
  int64_t nb = (L.np + kBlock - 1) / kBlock;
  if (nb > kNoAllocPartials) nb = kNoAllocPartials;
  k_mass_partial_na<T><<<(unsigned)nb, kBlock, 0, s>>>(static_cast<const T *>(d.f[src]), d.order, L.np, scr);
  k_mass_balance_na<<<1, kBlock, 0, s>>>(scr, nb, offset, m0, d.acc, out);
  return hipGetLastError();
}

}  // namespace

hipError_t noalloc_setup(double **addr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double *>(p);
  }
  if (addr) *addr = g_scratch[dev];
  return hipSuccess;
}

hipError_t launch_mass_balance_noalloc(const LaunchCfg &cfg, const Layout &L, const DevPtrs &d, int src,
                                       double offset, double m0, double *out, hipStream_t s) {
  double *scr = nullptr;
  hipError_t e = noalloc_setup(&scr);  // the address was looked up when the context was created
  if (e != hipSuccess) return e;
  switch (cfg.storage) {
    case HLB_F64: return mass_na<double>(L, d, src, offset, m0, scr, out, s);
    case HLB_F32_SHIFTED: return mass_na<float>(L, d, src, offset, m0, scr, out, s);
    case HLB_F16_SHIFTED: return mass_na<_Float16>(L, d, src, offset, m0, scr, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hlb
