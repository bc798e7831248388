// Halo exchange of the domain split without a receive buffer (Sec. 3.1's
// edge / mid-domain update, Sec. 3.2.3's exchange): the sender writes each
// exchanged population straight into the ghost slot of the receiving
// partition's population buffer that the receiver's next step pulls from,
// so there is neither a transfer nor an unpack pass.  On one GPU the peer
// buffer is ordinary device memory; between GPUs it would be the peer's
// buffer mapped over xGMI (an IPC handle).
#include "hlb_device.h"
#include "hlb_halo.h"

namespace hlb {
namespace {

using namespace dev;

// dst[elem[k]] = A[(pos[k], dir[k])] for k < n.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack_to_peer(const T *__restrict__ A, const int32_t *__restrict__ pos,
                                                         const int32_t *__restrict__ dir, int64_t n,
                                                         T *__restrict__ dst, const int64_t *__restrict__ elem) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) dst[elem[k]] = A[pidx(pos[k], dir[k])];
}

template <typename T>
hipError_t pack_impl(const void *src, const int32_t *pos, const int32_t *dir, int64_t n, void *dst,
                     const int64_t *elem, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  k_pack_to_peer<T><<<grid, kBlock, 0, s>>>(static_cast<const T *>(src), pos, dir, n, static_cast<T *>(dst), elem);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_to_peer(int storage, const void *src, const int32_t *pos, const int32_t *dir, int64_t n,
                               void *dst, const int64_t *elem, hipStream_t s) {
  switch (storage) {
    case HLB_F64: return pack_impl<double>(src, pos, dir, n, dst, elem, s);
    case HLB_F32_SHIFTED: return pack_impl<float>(src, pos, dir, n, dst, elem, s);
    case HLB_F16_SHIFTED: return pack_impl<_Float16>(src, pos, dir, n, dst, elem, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hlb
