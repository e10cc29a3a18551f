// exec.hpp -- launch interface of the gfx950 executor.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ec {

constexpr int kMaxBlocks = 32;  // input + output blocks of one stripe
constexpr int kTileBytes = 1024;  // bytes of each strip per wave (64 lanes x 16 B)
constexpr int kMaxParts = 8;      // row-split parts of whole output blocks
constexpr int kMaxRowParts = 32;  // row-split parts of single bit rows (or small groups)

// Kernel arguments of a single-stripe launch (passed by value).
struct ExecArgs {
  uint64_t blk[kMaxBlocks];  // n_in input block pointers, then the output block pointers
  const uint32_t *prog;      // device bytecode, padded with HALT words
  uint32_t n_in;             // input blocks
  uint32_t n_tiles;          // ceil(strip_len / kTileBytes)
  uint64_t strip_len;        // bytes per strip (block_bytes / 8), multiple of 16
  // Work item k runs tile tile_of(k, ...) (tile_order.hpp): with
  // seg_shift > 0 the strips are cut into 1 << seg_shift segments of
  // seg_tiles tiles, and each workgroup's 4 waves take 4 neighbouring tiles
  // of one segment, consecutive workgroups taking consecutive segments;
  // the identity when seg_shift = 0.
  uint32_t seg_shift, seg_mask, seg_tiles;
  // Row split: work item k runs part k % n_parts (the program at word
  // part_off[k % n_parts] of prog) on tile k / n_parts; n_parts = 1 and
  // part_off[0] = 0 run the whole program on every tile.
  uint32_t n_parts;
  uint32_t part_off[kMaxRowParts];
};

// One stripe of a batched launch (device memory, read-only during a launch).
struct StripeDesc {
  uint64_t blk[kMaxBlocks];      // input block pointers, then output block pointers
  const uint32_t *prog;          // the stripe's device image
  uint32_t n_blocks;             // input + output blocks
  uint32_t strip_len;            // bytes per strip
  uint32_t part_off[kMaxRowParts];  // word offset in prog of each part a work item may name
};                                  // (part 0 at offset 0: the whole program, when not split)

// Second word of a work item: first tile in the low bits, part above.
constexpr uint32_t kItemPartShift = 24;
constexpr uint32_t kItemTileMask = (1u << kItemPartShift) - 1;

// Arguments of the persistent batched kernel.
struct BatchArgs {
  const StripeDesc *stripes;
  const uint32_t *items;  // 2 words per work item: stripe index, tile | part << kItemPartShift
  uint32_t n_items;
  uint32_t tiles_per_item;  // consecutive tiles one work item covers
  uint32_t chunk;           // items taken per atomic add on the counter
  uint32_t *counter;        // next work item; reset to 0 by the launch itself
};

// Waves per SIMD the executor reaches for a slot budget: VGPRs per lane are
// 4 + 4K + a few of the kernel's own, allocated in granules of 8, out of 512.
inline int waves_per_simd(int slots) { return slots <= 24 ? 4 : slots <= 38 ? 3 : 2; }

// Reset the work counter and launch the persistent kernel for `slots`.
int batch_launch(int slots, const BatchArgs &a, int grid, hipStream_t stream);

// Launch the executor instance for `slots` register slots; 0 on success.
int exec_launch(int slots, const ExecArgs &a, int grid, hipStream_t stream);

// Device-to-device copy of `bytes` (a multiple of 16, 16-byte aligned) on a
// device of n_cus compute units.
int copy_launch(const void *src, void *dst, uint64_t bytes, int n_cus, hipStream_t stream);

// The data movement of one launch of the executor without a program: every
// tile reads all n_in input strips and writes all n_out output strips (the
// XOR of its inputs), a.blk holding the input then the output blocks, with
// the executor's tile order and grid.
int stream_launch(const ExecArgs &a, uint32_t n_out, int grid, hipStream_t stream);

}  // namespace ec
