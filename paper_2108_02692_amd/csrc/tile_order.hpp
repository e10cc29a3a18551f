// tile_order.hpp -- which tile of a stripe a launch's work item runs (device
// side; the host picks the segment fields, see exec.hpp ExecArgs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ec {

// Work items in groups of kTileGroup (one workgroup's waves): group g takes
// kTileGroup neighbouring tiles of segment g mod 2^seg_shift, the segments
// being 2^seg_shift equal runs of seg_tiles tiles.  With seg_shift = 0 this
// is the identity.  Needs seg_tiles % kTileGroup == 0 when seg_shift > 0.
constexpr uint32_t kTileGroup = 4;

__device__ __forceinline__ uint32_t tile_of(uint32_t kt, uint32_t seg_shift, uint32_t seg_mask, uint32_t seg_tiles) {
  const uint32_t g = kt / kTileGroup;
  return (g & seg_mask) * seg_tiles + (g >> seg_shift) * kTileGroup + kt % kTileGroup;
}

}  // namespace ec
