// bytecode.hpp -- the executor's record format.
//
// A program is a sequence of variable-length records, each two header words
// and n operand words (0 <= n <= 14), followed by 16 zero words (the executor
// reads a fixed 16-word window at every record).  The machine has one
// accumulator (16 B per lane) and K register slots; a record does, in this
// order, what its kind asks:
//
//   kind      WAIT  PULL  LD   STORE  then the run
//   RUN        -     -    -     -     (continuation: acc is kept)
//   INPUT      x     x    -     -
//   INPUT_LD   x     x    x     -
//   VALUE      -     x    -     -
//   STORE      -     x    -     x
//   LOAD       -     -    x     -
//   PREFETCH   (no register: 4 B per lane of strip (blk, j) into a scratch
//              register, so that the strip's lines are in the L2 cache when
//              its real load comes; counts as a memory operation for WAIT)
//   HALT       end of the program
//
//   WAIT   s_waitcnt vmcnt(wait): the pulled slot's load has landed
//   PULL   acc = slot[pull]
//   LD     slot[ld] = 16 B per lane of strip (blk, j) of this tile
//   STORE  strip (blk, j) of this tile = acc
//   run    slot[op] ^= acc for every operand (an operand equal to the pulled
//          slot clears it, which is how accumulators are returned to zero)
//
// Header word 0:  [7:0] 4*pull slot   [11:9] kind   [18:12] record bytes
//                 (8 + 4n)   [27:19] byte offset of the run's entry in the
//                 unrolled 14-step run table, (14 - n) * 20
// Header word 1:  [8:0] 8*wait   [18:9] 16*ld slot   [23:19] blk   [26:24] j
// Operand words:  4*slot.
// Every other bit is zero.  The scaled fields are the byte offsets the
// executor's computed jumps use directly.
#pragma once

#include <cstdint>

namespace ec {
namespace bc {

enum Kind : uint32_t { RUN = 0, INPUT = 1, INPUT_LD = 2, VALUE = 3, STORE = 4, LOAD = 5, HALT = 6, PREFETCH = 7 };

constexpr int kMaxOps = 14;       // operands per record
constexpr int kWindow = 16;       // words the executor reads per record
constexpr int kRunStepBytes = 20; // s_set_gpr_idx_on + 4 x v_xor_b32 (VOP2)
constexpr int kMaxWait = 63;      // vmcnt field

constexpr uint32_t h0(uint32_t kind, uint32_t pull_slot, uint32_t n) {
  return (4u * pull_slot) | (kind << 9) | ((8u + 4u * n) << 12) | (((uint32_t)kMaxOps - n) * kRunStepBytes << 19);
}
constexpr uint32_t h1(uint32_t wait, uint32_t ld_slot, uint32_t blk, uint32_t j) {
  return (8u * wait) | ((16u * ld_slot) << 9) | (blk << 19) | (j << 24);
}
constexpr uint32_t h0_kind(uint32_t w) { return (w >> 9) & 7u; }
constexpr uint32_t h0_pull(uint32_t w) { return (w & 0xffu) >> 2; }
constexpr uint32_t h0_bytes(uint32_t w) { return (w >> 12) & 0x7fu; }
constexpr uint32_t h0_runoff(uint32_t w) { return (w >> 19) & 0x1ffu; }
constexpr uint32_t h1_wait(uint32_t w) { return (w & 0x1ffu) >> 3; }
constexpr uint32_t h1_ld(uint32_t w) { return ((w >> 9) & 0x3ffu) >> 4; }
constexpr uint32_t h1_blk(uint32_t w) { return (w >> 19) & 0x1fu; }
constexpr uint32_t h1_j(uint32_t w) { return (w >> 24) & 7u; }

}  // namespace bc
}  // namespace ec
