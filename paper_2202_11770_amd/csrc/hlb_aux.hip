// Small auxiliary kernels of the runtime: checks of caller-supplied device
// arrays, and moves of per-site values between the caller's site order and
// the library's positions.  None of them is on the path of a step.
#include "hlb_aux.h"

namespace hlb {
namespace {

constexpr int kAuxBlock = 256;

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kAuxBlock - 1) / kAuxBlock;
  return (unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b));
}

// flag := 1 if any value breaks the rule of `mode` (NaN breaks every rule).
__global__ void k_check_values(const double *__restrict__ v, int64_t n, int mode, int32_t *flag) {
  bool bad = false;
  for (int64_t k = (int64_t)blockIdx.x * kAuxBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kAuxBlock) {
    const double x = v[k];
    if (mode == kCheckFinite) bad |= !__builtin_isfinite(x);
    else if (mode == kCheckPositive) bad |= !(__builtin_isfinite(x) && x > 0.0);
    else bad |= !(x >= 0.0 && x <= 1.0);
  }
  if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ void k_zero_flag(int32_t *flag) { *flag = 0; }

__global__ void k_from_caller(const double *__restrict__ caller, const int32_t *__restrict__ order, int64_t np,
                              double *__restrict__ pos) {
  for (int64_t p = (int64_t)blockIdx.x * kAuxBlock + threadIdx.x; p < np; p += (int64_t)gridDim.x * kAuxBlock) {
    const int32_t x = order[p];
    pos[p] = x >= 0 ? caller[x] : 0.0;
  }
}

__global__ void k_to_caller(const double *__restrict__ pos, const int32_t *__restrict__ order, int64_t np,
                            double *__restrict__ caller) {
  for (int64_t p = (int64_t)blockIdx.x * kAuxBlock + threadIdx.x; p < np; p += (int64_t)gridDim.x * kAuxBlock) {
    const int32_t x = order[p];
    if (x >= 0) caller[x] = pos[p];
  }
}

}  // namespace

hipError_t launch_check_values(const double *v, int64_t n, int mode, int32_t *flag, hipStream_t s) {
  k_zero_flag<<<1, 1, 0, s>>>(flag);
  if (n > 0) k_check_values<<<grid_for(n), kAuxBlock, 0, s>>>(v, n, mode, flag);
  return hipGetLastError();
}

hipError_t launch_from_caller(const double *caller, const int32_t *order, int64_t np, double *pos, hipStream_t s) {
  k_from_caller<<<grid_for(np), kAuxBlock, 0, s>>>(caller, order, np, pos);
  return hipGetLastError();
}

hipError_t launch_to_caller(const double *pos, const int32_t *order, int64_t np, double *caller, hipStream_t s) {
  k_to_caller<<<grid_for(np), kAuxBlock, 0, s>>>(pos, order, np, caller);
  return hipGetLastError();
}

}  // namespace hlb
