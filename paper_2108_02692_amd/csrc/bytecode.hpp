// bytecode.hpp -- device bytecode of a compiled XOR program.
//
// One program runs once per tile (a 16-byte-per-lane, 1 KiB-per-wave slice
// of every strip).  The executor holds K register slots of 16 bytes per lane
// and one 16-byte accumulator.  The compiler first produces a linear stream
// of micro-ops, then packs it into blocks; the device only sees blocks.
//
// Linear micro-ops (compiler-internal):
//   OPERAND s        acc ^= slot[s]
//   END flags        PUT: slot[d] = acc; STORE: output strip o = acc;
//                    KEEP: keep acc (else acc = 0 afterwards)
//   LD s, c          slot[s] <- input strip c (asynchronous)
//   WAIT n           wait until at most n vector memory ops are outstanding
//   HALT             end of the tile
//
// Device block (2 header words + n operand words, n <= 14), executed as
//   [LD] [WAIT] n x OPERAND [PUT] [STORE] [CLEAR] [HALT]:
//   H0: bits 3:0 n | bit 4 LD | bits 10:5 LD slot | bits 21:11 LD strip |
//       bit 22 WAIT | bits 28:23 WAIT count
//   H1: bit 0 PUT | bit 1 STORE | bit 2 CLEAR | bit 3 HALT |
//       bits 10:5 PUT slot | bits 21:11 STORE strip
//   operand word: 4 * slot (bits 7:0), the VGPR offset of the slot.
// Input strip c is strip c % 8 of input argument c / 8; output strip o is
// strip o % 8 of output argument o / 8.
#pragma once

#include <cstdint>
#include <vector>

namespace ec {
namespace bc {

// ---- linear micro-ops
enum Kind : uint8_t { OPERAND, END, LD, WAIT, HALT };
struct Micro {
  Kind kind;
  uint8_t flags;   // END: kEndPut | kEndStore | kEndKeep
  int16_t slot;    // OPERAND / LD / END-put slot
  int16_t strip;   // LD input strip / END-store output strip
  int16_t count;   // WAIT count
};
constexpr uint8_t kEndPut = 1, kEndStore = 2, kEndKeep = 4;

// ---- device blocks
constexpr int kMaxOperands = 14;
constexpr int kWindow = 16;       // words the device reads per block
constexpr int kMaxStrip = 2047;   // 11-bit strip fields
constexpr int kMaxSlot = 63;      // 6-bit slot fields
constexpr int kMaxVmcnt = 63;     // 6-bit vector memory counter

constexpr uint32_t H0_N = 0xFu, H0_LD = 1u << 4, H0_WAIT = 1u << 22;
constexpr uint32_t H1_PUT = 1u, H1_STORE = 2u, H1_CLEAR = 4u, H1_HALT = 8u;

constexpr uint32_t h0_ld_slot(uint32_t h) { return (h >> 5) & 63u; }
constexpr uint32_t h0_ld_strip(uint32_t h) { return (h >> 11) & 0x7FFu; }
constexpr uint32_t h0_wait(uint32_t h) { return (h >> 23) & 63u; }
constexpr uint32_t h1_put_slot(uint32_t h) { return (h >> 5) & 63u; }
constexpr uint32_t h1_store_strip(uint32_t h) { return (h >> 11) & 0x7FFu; }

// Pack a linear micro-op stream into device blocks (terminated by HALT,
// followed by kWindow zero words so the device may read ahead).
std::vector<uint32_t> pack(const std::vector<Micro> &ops);

}  // namespace bc
}  // namespace ec
