// Measurement aid: a plain device-to-device copy, the practical ceiling of
// HBM bandwidth against which the step kernel is read (and, at a known
// size, the reference for scaling the HBM byte counters).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hlb.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const f4 *__restrict__ a, f4 *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

}  // namespace

extern "C" hlb_status hlb_copy_bandwidth(int64_t bytes, int32_t reps, double *gbs) {
  if (bytes < (1 << 20) || bytes % 16 != 0 || reps < 1 || !gbs) return HLB_EINVAL;
  void *a = nullptr, *b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hlb_status st = HLB_EDEVICE;
  const int64_t n = bytes / 16;
  const unsigned grid = (unsigned)((n + 255) / 256);
  float ms = 0.f;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    st = HLB_ENOMEM;
    goto done;
  }
  if (hipMemset(a, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    goto done;
  k_copy<<<grid, 256>>>(static_cast<const f4 *>(a), static_cast<f4 *>(b), n);
  if (hipEventRecord(e0, nullptr) != hipSuccess) goto done;
  for (int r = 0; r < reps; ++r) k_copy<<<grid, 256>>>(static_cast<const f4 *>(a), static_cast<f4 *>(b), n);
  if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
    goto done;
  *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
  st = HLB_OK;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  (void)hipGetLastError();
  return st;
}
