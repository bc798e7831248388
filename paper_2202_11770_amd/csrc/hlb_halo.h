// Launcher of the direct halo pack (hlb_halo.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hlb {

// dst[elem[k]] := population dir[k] of position pos[k] in the population
// buffer src (tiled, of the storage type), k < n; dst is a peer partition's
// population buffer and elem its element indices of the receiving ghost
// slots.  Asynchronous on s.
hipError_t launch_pack_to_peer(int storage, const void *src, const int32_t *pos, const int32_t *dir, int64_t n,
                               void *dst, const int64_t *elem, hipStream_t s);

}  // namespace hlb
