// bytecode.hpp -- device bytecode of a compiled XOR program.
//
// One program runs once per tile (a 16-byte-per-lane, 1 KiB-per-wave slice
// of every strip).  The executor holds K register slots of 16 bytes per lane
// and one 16-byte accumulator (acc).  The compiler first produces a linear
// stream of micro-ops, then packs it into fixed 16-word blocks; the device
// only sees blocks.
//
// Micro-ops:
//   PULL s        acc ^= slot[s]
//   PUSH s        slot[s] ^= acc
//   PUSHSET s     slot[s] = acc
//   PUT s         slot[s] = acc
//   STORE o       output strip o <- acc
//   CLEAR         acc = 0
//   LD s, c       slot[s] <- input strip c (asynchronous)
//   WAIT n        wait until at most n vector memory ops are outstanding
//   HALT          end of the tile
//
// Device block: 16 words.  Word 0 (H0) and word 1 (H1) are headers; pull
// operands occupy words 2 .. 2+np-1 and push operands words 16-nq .. 15
// (np + nq <= 14).  A block executes, in this order:
//   [LD] [WAIT] np x PULL [PUT] [STORE] nq x PUSH (or PUSHSET) [CLEAR] [HALT]
//   H0: bits 3:0 np | bits 7:4 nq | bit 8 LD | bits 14:9 LD slot |
//       bits 25:15 LD strip | bit 26 WAIT | bit 27 push runs set (PUSHSET)
//   H1: bits 5:0 WAIT count | bit 6 PUT | bits 12:7 PUT slot | bit 13 STORE |
//       bits 24:14 STORE strip | bit 25 CLEAR | bit 26 HALT
//   operand word: 4 * slot (bits 7:0), the VGPR offset of the slot.
// Input strip c is strip c % 8 of input argument c / 8; output strip o is
// strip o % 8 of output argument o / 8.
#pragma once

#include <cstdint>
#include <vector>

namespace ec {
namespace bc {

// ---- linear micro-ops
enum Kind : uint8_t { PULL, PUSH, PUSHSET, PUT, STORE, CLEAR, LD, WAIT, HALT };
struct Micro {
  Kind kind;
  int16_t slot;   // PULL / PUSH / PUSHSET / PUT / LD
  int16_t strip;  // LD input strip / STORE output strip
  int16_t count;  // WAIT
};

// ---- device blocks
constexpr int kBlockWords = 16;
constexpr int kMaxOperands = 14;  // np + nq
constexpr int kMaxStrip = 2047;   // 11-bit strip fields
constexpr int kMaxSlot = 63;      // 6-bit slot fields
constexpr int kMaxVmcnt = 63;     // 6-bit vector memory counter

constexpr uint32_t H0_LD = 1u << 8, H0_WAIT = 1u << 26, H0_SET = 1u << 27;
constexpr uint32_t H1_PUT = 1u << 6, H1_STORE = 1u << 13, H1_CLEAR = 1u << 25, H1_HALT = 1u << 26;

constexpr uint32_t h0_np(uint32_t h) { return h & 15u; }
constexpr uint32_t h0_nq(uint32_t h) { return (h >> 4) & 15u; }
constexpr uint32_t h0_ld_slot(uint32_t h) { return (h >> 9) & 63u; }
constexpr uint32_t h0_ld_strip(uint32_t h) { return (h >> 15) & 0x7FFu; }
constexpr uint32_t h1_wait(uint32_t h) { return h & 63u; }
constexpr uint32_t h1_put_slot(uint32_t h) { return (h >> 7) & 63u; }
constexpr uint32_t h1_store_strip(uint32_t h) { return (h >> 14) & 0x7FFu; }

// Pack a linear micro-op stream into device blocks; the last block carries
// HALT and one zero block follows, so the device may prefetch past HALT.
std::vector<uint32_t> pack(const std::vector<Micro> &ops);

}  // namespace bc
}  // namespace ec
