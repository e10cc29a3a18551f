// exec.hip -- gfx950 executor for compiled XOR programs.
//
// One wave runs the whole program on one tile: 64 lanes x 16 bytes = 1 KiB of
// every input and output strip (the blocked loop of Sec. 6.1, the tile being
// the paper's block size).  Values live in K register slots of 16 bytes per
// lane pinned to v[4 : 4+4K); the accumulator is pinned to v[0:3].
//  * A block's operands are XORed into the accumulator by a computed jump
//    into an unrolled run of VGPR-indexed XORs (s_set_gpr_idx_on with index
//    4*slot, then four v_xor_b32): temporaries stay in registers and never
//    reach memory (the deforestation of Sec. 5, with registers as the
//    pebbles of Sec. 6).
//  * Strip loads (global_load_dwordx4: 16 B per lane, 1 KiB per wave, fully
//    coalesced) land directly in their slot through a jump table; stores
//    write the accumulator.  Waits are the compiler's exact vmcnt counts,
//    dispatched through a second jump table.
//  * Blocks are read through the scalar cache, the next one prefetched while
//    the current one runs.
// The bytecode is validated on the host; the device trusts every field.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bytecode.hpp"
#include "exec.hpp"

namespace ec {

typedef uint32_t v32u __attribute__((ext_vector_type(32)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Pinned register groups: the accumulator and K/8 groups of 8 slots.
#define EC_G2 "+{v[0:3]}"(acc), "+{v[4:35]}"(g0), "+{v[36:67]}"(g1)
#define EC_G3 EC_G2, "+{v[68:99]}"(g2)
#define EC_G4 EC_G3, "+{v[100:131]}"(g3)
#define EC_G5 EC_G4, "+{v[132:163]}"(g4)
#define EC_G6 EC_G5, "+{v[164:195]}"(g5)

// An asm statement that may read or write the accumulator and every slot.
#define EC_SLOT_ASM(K, CODE, ...)                                        \
  do {                                                                   \
    if constexpr (K == 16) asm volatile(CODE : EC_G2 : __VA_ARGS__);     \
    else if constexpr (K == 24) asm volatile(CODE : EC_G3 : __VA_ARGS__); \
    else if constexpr (K == 32) asm volatile(CODE : EC_G4 : __VA_ARGS__); \
    else if constexpr (K == 40) asm volatile(CODE : EC_G5 : __VA_ARGS__); \
    else asm volatile(CODE : EC_G6 : __VA_ARGS__);                       \
  } while (0)

// Defines the pinned registers (no initial value except acc = 0), so the
// compiler never sees two groups holding one value and never copies them.
#define EC_G2_OUT "={v[0:3]}"(acc), "={v[4:35]}"(g0), "={v[36:67]}"(g1)
#define EC_G3_OUT EC_G2_OUT, "={v[68:99]}"(g2)
#define EC_G4_OUT EC_G3_OUT, "={v[100:131]}"(g3)
#define EC_G5_OUT EC_G4_OUT, "={v[132:163]}"(g4)
#define EC_G6_OUT EC_G5_OUT, "={v[164:195]}"(g5)
#define EC_ZERO_ACC "v_mov_b32_e32 v0, 0\n\tv_mov_b32_e32 v1, 0\n\tv_mov_b32_e32 v2, 0\n\tv_mov_b32_e32 v3, 0"
#define EC_SLOT_INIT(K)                                              \
  do {                                                               \
    if constexpr (K == 16) asm volatile(EC_ZERO_ACC : EC_G2_OUT);    \
    else if constexpr (K == 24) asm volatile(EC_ZERO_ACC : EC_G3_OUT); \
    else if constexpr (K == 32) asm volatile(EC_ZERO_ACC : EC_G4_OUT); \
    else if constexpr (K == 40) asm volatile(EC_ZERO_ACC : EC_G5_OUT); \
    else asm volatile(EC_ZERO_ACC : EC_G6_OUT);                      \
  } while (0)

// Groups as inputs only (the statement reads slots but writes only acc).
#define EC_GI2 "{v[4:35]}"(g0), "{v[36:67]}"(g1)
#define EC_GI3 EC_GI2, "{v[68:99]}"(g2)
#define EC_GI4 EC_GI3, "{v[100:131]}"(g3)
#define EC_GI5 EC_GI4, "{v[132:163]}"(g4)
#define EC_GI6 EC_GI5, "{v[164:195]}"(g5)
#define EC_ACC_ASM(K, CODE, ...)                                                    \
  do {                                                                              \
    if constexpr (K == 16) asm volatile(CODE : "+{v[0:3]}"(acc) : EC_GI2, __VA_ARGS__); \
    else if constexpr (K == 24) asm volatile(CODE : "+{v[0:3]}"(acc) : EC_GI3, __VA_ARGS__); \
    else if constexpr (K == 32) asm volatile(CODE : "+{v[0:3]}"(acc) : EC_GI4, __VA_ARGS__); \
    else if constexpr (K == 40) asm volatile(CODE : "+{v[0:3]}"(acc) : EC_GI5, __VA_ARGS__); \
    else asm volatile(CODE : "+{v[0:3]}"(acc) : EC_GI6, __VA_ARGS__);             \
  } while (0)

#define SLOT_PARAMS v4u &acc, v32u &g0, v32u &g1, v32u &g2, v32u &g3, v32u &g4, v32u &g5
#define SLOT_ARGS acc, g0, g1, g2, g3, g4, g5

struct Win {
  uint32_t w[bc::kBlockWords];
};

// The bytecode is read-only while a kernel runs: reading it through the
// constant address space lets every block come through the scalar cache
// (s_load_dwordx16), whatever the surrounding asm statements may touch.
typedef const __attribute__((address_space(4))) Win *ConstWinPtr;
__device__ __forceinline__ Win load_block(const uint32_t *prog, uint32_t pc) {
  ConstWinPtr p = (ConstWinPtr)(uintptr_t)(prog + pc);
  Win r;
#pragma unroll
  for (int i = 0; i < bc::kBlockWords; ++i) r.w[i] = p->w[i];
  return r;
}

template <int K>
__device__ __forceinline__ void issue_load(uint32_t slot, uint32_t voff, uint64_t base, SLOT_PARAMS);

template <>
__device__ __forceinline__ void issue_load<16>(uint32_t slot, uint32_t voff, uint64_t base, SLOT_PARAMS) {
  EC_SLOT_ASM(16,
      "s_nop 4\n\t"
      "s_getpc_b64 s[80:81]\n"
      "1:\n\t"
      "s_lshl_b32 s82, %[slot], 4\n\t"
      "s_add_u32 s82, s82, 2f-1b\n\t"
      "s_add_u32 s80, s80, s82\n\t"
      "s_addc_u32 s81, s81, 0\n\t"
      "s_setpc_b64 s[80:81]\n"
      "2:\n\t"
      "global_load_dwordx4 v[4:7], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[8:11], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[12:15], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[16:19], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[20:23], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[24:27], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[28:31], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[32:35], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[36:39], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[40:43], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[44:47], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[48:51], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[52:55], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[56:59], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[60:63], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[64:67], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "3:",
      [slot] "s"(slot), [off] "v"(voff), [base] "s"(base) : "s80", "s81", "s82", "scc");
}

template <>
__device__ __forceinline__ void issue_load<24>(uint32_t slot, uint32_t voff, uint64_t base, SLOT_PARAMS) {
  EC_SLOT_ASM(24,
      "s_nop 4\n\t"
      "s_getpc_b64 s[80:81]\n"
      "1:\n\t"
      "s_lshl_b32 s82, %[slot], 4\n\t"
      "s_add_u32 s82, s82, 2f-1b\n\t"
      "s_add_u32 s80, s80, s82\n\t"
      "s_addc_u32 s81, s81, 0\n\t"
      "s_setpc_b64 s[80:81]\n"
      "2:\n\t"
      "global_load_dwordx4 v[4:7], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[8:11], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[12:15], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[16:19], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[20:23], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[24:27], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[28:31], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[32:35], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[36:39], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[40:43], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[44:47], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[48:51], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[52:55], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[56:59], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[60:63], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[64:67], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[68:71], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[72:75], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[76:79], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[80:83], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[84:87], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[88:91], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[92:95], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[96:99], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "3:",
      [slot] "s"(slot), [off] "v"(voff), [base] "s"(base) : "s80", "s81", "s82", "scc");
}

template <>
__device__ __forceinline__ void issue_load<32>(uint32_t slot, uint32_t voff, uint64_t base, SLOT_PARAMS) {
  EC_SLOT_ASM(32,
      "s_nop 4\n\t"
      "s_getpc_b64 s[80:81]\n"
      "1:\n\t"
      "s_lshl_b32 s82, %[slot], 4\n\t"
      "s_add_u32 s82, s82, 2f-1b\n\t"
      "s_add_u32 s80, s80, s82\n\t"
      "s_addc_u32 s81, s81, 0\n\t"
      "s_setpc_b64 s[80:81]\n"
      "2:\n\t"
      "global_load_dwordx4 v[4:7], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[8:11], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[12:15], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[16:19], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[20:23], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[24:27], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[28:31], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[32:35], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[36:39], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[40:43], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[44:47], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[48:51], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[52:55], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[56:59], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[60:63], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[64:67], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[68:71], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[72:75], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[76:79], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[80:83], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[84:87], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[88:91], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[92:95], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[96:99], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[100:103], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[104:107], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[108:111], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[112:115], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[116:119], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[120:123], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[124:127], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[128:131], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "3:",
      [slot] "s"(slot), [off] "v"(voff), [base] "s"(base) : "s80", "s81", "s82", "scc");
}

template <>
__device__ __forceinline__ void issue_load<40>(uint32_t slot, uint32_t voff, uint64_t base, SLOT_PARAMS) {
  EC_SLOT_ASM(40,
      "s_nop 4\n\t"
      "s_getpc_b64 s[80:81]\n"
      "1:\n\t"
      "s_lshl_b32 s82, %[slot], 4\n\t"
      "s_add_u32 s82, s82, 2f-1b\n\t"
      "s_add_u32 s80, s80, s82\n\t"
      "s_addc_u32 s81, s81, 0\n\t"
      "s_setpc_b64 s[80:81]\n"
      "2:\n\t"
      "global_load_dwordx4 v[4:7], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[8:11], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[12:15], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[16:19], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[20:23], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[24:27], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[28:31], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[32:35], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[36:39], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[40:43], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[44:47], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[48:51], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[52:55], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[56:59], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[60:63], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[64:67], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[68:71], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[72:75], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[76:79], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[80:83], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[84:87], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[88:91], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[92:95], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[96:99], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[100:103], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[104:107], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[108:111], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[112:115], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[116:119], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[120:123], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[124:127], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[128:131], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[132:135], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[136:139], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[140:143], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[144:147], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[148:151], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[152:155], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[156:159], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[160:163], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "3:",
      [slot] "s"(slot), [off] "v"(voff), [base] "s"(base) : "s80", "s81", "s82", "scc");
}

template <>
__device__ __forceinline__ void issue_load<48>(uint32_t slot, uint32_t voff, uint64_t base, SLOT_PARAMS) {
  EC_SLOT_ASM(48,
      "s_nop 4\n\t"
      "s_getpc_b64 s[80:81]\n"
      "1:\n\t"
      "s_lshl_b32 s82, %[slot], 4\n\t"
      "s_add_u32 s82, s82, 2f-1b\n\t"
      "s_add_u32 s80, s80, s82\n\t"
      "s_addc_u32 s81, s81, 0\n\t"
      "s_setpc_b64 s[80:81]\n"
      "2:\n\t"
      "global_load_dwordx4 v[4:7], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[8:11], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[12:15], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[16:19], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[20:23], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[24:27], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[28:31], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[32:35], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[36:39], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[40:43], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[44:47], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[48:51], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[52:55], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[56:59], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[60:63], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[64:67], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[68:71], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[72:75], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[76:79], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[80:83], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[84:87], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[88:91], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[92:95], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[96:99], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[100:103], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[104:107], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[108:111], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[112:115], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[116:119], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[120:123], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[124:127], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[128:131], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[132:135], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[136:139], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[140:143], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[144:147], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[148:151], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[152:155], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[156:159], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[160:163], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[164:167], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[168:171], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[172:175], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[176:179], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[180:183], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[184:187], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[188:191], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "global_load_dwordx4 v[192:195], %[off], %[base]\n\ts_branch 3f\n\ts_nop 0\n\t"
      "3:",
      [slot] "s"(slot), [off] "v"(voff), [base] "s"(base) : "s80", "s81", "s82", "scc");
}

// s_waitcnt vmcnt(n) for a data-dependent n, through a jump table.  Touches
// no register the compiler tracks.
__device__ __forceinline__ void wait_vm(uint32_t n) {
  asm volatile(
      "s_getpc_b64 s[80:81]\n"
      "1:\n\t"
      "s_lshl_b32 s82, %[n], 3\n\t"
      "s_add_u32 s82, s82, 2f-1b\n\t"
      "s_add_u32 s80, s80, s82\n\t"
      "s_addc_u32 s81, s81, 0\n\t"
      "s_setpc_b64 s[80:81]\n"
      "2:\n\t"
      "s_waitcnt vmcnt(0)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(1)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(2)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(3)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(4)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(5)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(6)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(7)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(8)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(9)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(10)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(11)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(12)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(13)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(14)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(15)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(16)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(17)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(18)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(19)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(20)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(21)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(22)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(23)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(24)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(25)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(26)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(27)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(28)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(29)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(30)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(31)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(32)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(33)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(34)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(35)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(36)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(37)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(38)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(39)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(40)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(41)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(42)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(43)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(44)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(45)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(46)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(47)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(48)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(49)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(50)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(51)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(52)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(53)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(54)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(55)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(56)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(57)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(58)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(59)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(60)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(61)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(62)\n\ts_branch 3f\n\t"
      "s_waitcnt vmcnt(63)\n\ts_branch 3f\n\t"
      "3:"
      :: [n] "s"(n) : "s80", "s81", "s82", "scc");
}

// A run of n operand steps, entered by a computed jump that skips 14 - n of
// the 14 unrolled 20-byte steps (each: s_set_gpr_idx_on + 4 VALU ops).
#define EC_JUMP(L1, L2, SKIP)                          \
  "s_getpc_b64 s[80:81]\n" L1 ":\n\t"                  \
  "s_mul_i32 s82, " SKIP ", 20\n\t"                    \
  "s_add_u32 s82, s82, " L2 "f-" L1 "b\n\t"            \
  "s_add_u32 s80, s80, s82\n\t"                        \
  "s_addc_u32 s81, s81, 0\n\t"                         \
  "s_setpc_b64 s[80:81]\n" L2 ":\n\t"
#define EC_WORDS                                                                                   \
  [w2] "s"(W.w[2]), [w3] "s"(W.w[3]), [w4] "s"(W.w[4]), [w5] "s"(W.w[5]), [w6] "s"(W.w[6]),         \
  [w7] "s"(W.w[7]), [w8] "s"(W.w[8]), [w9] "s"(W.w[9]), [w10] "s"(W.w[10]), [w11] "s"(W.w[11]),     \
  [w12] "s"(W.w[12]), [w13] "s"(W.w[13]), [w14] "s"(W.w[14]), [w15] "s"(W.w[15])

// acc ^= slot[w] for the n pull words (words 2 .. 2+n-1); n = 0 jumps past
// every step.
template <int K>
__device__ __forceinline__ void pull_run(const Win &W, uint32_t n, SLOT_PARAMS) {
  const uint32_t skip = __builtin_amdgcn_readfirstlane((uint32_t)bc::kMaxOperands - n);
  EC_ACC_ASM(K, EC_JUMP("1", "2", "%[skip]") "s_set_gpr_idx_on %[w15], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w14], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w13], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w12], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w11], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w10], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w9], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w8], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w7], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w6], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w5], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w4], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w3], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t"
                "s_set_gpr_idx_on %[w2], gpr_idx(SRC0)\n\t"
                "v_xor_b32_e32 v0, v4, v0\n\tv_xor_b32_e32 v1, v5, v1\n\tv_xor_b32_e32 v2, v6, v2\n\tv_xor_b32_e32 v3, v7, v3\n\t" "s_set_gpr_idx_off",
             [skip] "s"(skip), EC_WORDS : "s80", "s81", "s82", "scc");
}

// For the n push words (words 16-n .. 15): slot[w] ^= acc, or slot[w] = acc
// when `set` is nonzero.  One asm statement for both forms, so the register
// allocator sees a single producer of the slot registers.
template <int K>
__device__ __forceinline__ void push_run(const Win &W, uint32_t n, uint32_t set, SLOT_PARAMS) {
  const uint32_t skip = __builtin_amdgcn_readfirstlane((uint32_t)bc::kMaxOperands - n);
  const uint32_t is_set = __builtin_amdgcn_readfirstlane(set);
  EC_SLOT_ASM(K,
              "s_cmp_lg_u32 %[set], 0\n\t"
              "s_cbranch_scc1 5f\n\t"
              EC_JUMP("1", "2", "%[skip]") "s_set_gpr_idx_on %[w2], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w3], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w4], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w5], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w6], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w7], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w8], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w9], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w10], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w11], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w12], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w13], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w14], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t"
                "s_set_gpr_idx_on %[w15], gpr_idx(SRC0,DST)\n\t"
                "v_xor_b32_e32 v4, v4, v0\n\tv_xor_b32_e32 v5, v5, v1\n\tv_xor_b32_e32 v6, v6, v2\n\tv_xor_b32_e32 v7, v7, v3\n\t" "s_set_gpr_idx_off\n\t"
              "s_branch 6f\n"
              "5:\n\t"
              EC_JUMP("3", "4", "%[skip]") "s_set_gpr_idx_on %[w2], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w3], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w4], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w5], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w6], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w7], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w8], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w9], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w10], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w11], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w12], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w13], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w14], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_on %[w15], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\tv_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t" "s_set_gpr_idx_off\n"
              "6:",
              [skip] "s"(skip), [set] "s"(is_set), EC_WORDS : "s80", "s81", "s82", "scc");
}

__device__ __forceinline__ uint64_t strip_base(uint32_t tab_lo, uint32_t tab_hi, uint32_t blk, uint32_t strip,
                                               uint32_t strip_len, uint64_t toff) {
  const uint64_t p = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)tab_hi, (int)blk) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane((int)tab_lo, (int)blk);
  return p + (uint64_t)(strip * strip_len) + toff;
}

// Runs block `W` and prefetches the next one (blocks have a fixed size, so
// its address is known at once); returns true at HALT.
template <int K>
__device__ __forceinline__ bool run_block(const uint32_t *__restrict__ prog, const Win &W, uint32_t &pc, Win &next,
                                          uint32_t voff, uint32_t tab_lo, uint32_t tab_hi, uint32_t n_in,
                                          uint32_t strip_len, uint64_t toff, SLOT_PARAMS) {
  const uint32_t h0 = W.w[0], h1 = W.w[1];
  pc += bc::kBlockWords;
  next = load_block(prog, pc);
  if (h0 & bc::H0_LD) {
    const uint32_t c = bc::h0_ld_strip(h0);
    // slot clamped so the jump stays inside the table (the host validates it)
    issue_load<K>(__builtin_amdgcn_readfirstlane(min(bc::h0_ld_slot(h0), (uint32_t)(K - 1))), voff,
                  strip_base(tab_lo, tab_hi, c >> 3, c & 7u, strip_len, toff), SLOT_ARGS);
  }
  if (h0 & bc::H0_WAIT) wait_vm(__builtin_amdgcn_readfirstlane(bc::h1_wait(h1)));  // 6-bit field: always in the table
  // run lengths clamped to the 14 unrolled steps
  const uint32_t np = min(bc::h0_np(h0), (uint32_t)bc::kMaxOperands);
  const uint32_t nq = min(bc::h0_nq(h0), (uint32_t)bc::kMaxOperands);
  pull_run<K>(W, np, SLOT_ARGS);
  if (h1 & bc::H1_PUT) {
    EC_SLOT_ASM(K,
                "s_set_gpr_idx_on %[i], gpr_idx(DST)\n\t"
                "v_mov_b32_e32 v4, v0\n\tv_mov_b32_e32 v5, v1\n\t"
                "v_mov_b32_e32 v6, v2\n\tv_mov_b32_e32 v7, v3\n\t"
                "s_set_gpr_idx_off",
                [i] "s"(__builtin_amdgcn_readfirstlane(min(bc::h1_put_slot(h1), (uint32_t)(K - 1)) * 4u)));
  }
  if (h1 & bc::H1_STORE) {
    const uint32_t o = bc::h1_store_strip(h1);
    const uint64_t base = strip_base(tab_lo, tab_hi, n_in + (o >> 3), o & 7u, strip_len, toff);
    // s_nop 4: the base may come from v_readlane; s_nop 1: one wait state
    // before a VALU may overwrite the data registers of a 16-byte store.
    asm volatile("s_nop 4\n\tglobal_store_dwordx4 %[off], v[0:3], %[base]\n\ts_nop 1"
                 :: "{v[0:3]}"(acc), [off] "v"(voff), [base] "s"(base));
  }
  push_run<K>(W, nq, h0 & bc::H0_SET, SLOT_ARGS);
  if (h1 & bc::H1_CLEAR) asm volatile(EC_ZERO_ACC : "+{v[0:3]}"(acc));
  return (h1 & bc::H1_HALT) != 0;
}

template <int K>
__device__ __forceinline__ void run_tile(const uint32_t *__restrict__ prog, uint32_t voff, uint32_t tab_lo,
                                         uint32_t tab_hi, uint32_t n_in, uint32_t strip_len, uint64_t toff,
                                         SLOT_PARAMS) {
  uint32_t pc = 0;
  Win A = load_block(prog, 0), B;
  // Two windows used in turn, so no copy between blocks.
  for (;;) {
    if (run_block<K>(prog, A, pc, B, voff, tab_lo, tab_hi, n_in, strip_len, toff, SLOT_ARGS)) break;
    if (run_block<K>(prog, B, pc, A, voff, tab_lo, tab_hi, n_in, strip_len, toff, SLOT_ARGS)) break;
  }
}

template <int K>
__global__ void __launch_bounds__(256) slp_exec_kernel(ExecArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  // wave index as a scalar: every per-tile address below is wave-uniform
  const uint32_t wave = blockIdx.x * 4u + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t n_waves = gridDim.x * 4u;
  // Block pointer table: lane b holds the pointer of block b.
  uint32_t tab_lo = 0, tab_hi = 0;
#pragma unroll
  for (int b = 0; b < kMaxBlocks; ++b)
    if ((int)lane == b) {
      tab_lo = (uint32_t)a.blk[b];
      tab_hi = (uint32_t)(a.blk[b] >> 32);
    }
  const uint32_t voff = lane * 16u;
  // the slot registers come to life here, after the prologue's temporaries
  v4u acc;
  v32u g0, g1, g2, g3, g4, g5;
  EC_SLOT_INIT(K);
  for (uint32_t tile = wave; tile < a.n_tiles; tile += n_waves) {
    const uint64_t toff = (uint64_t)tile * kTileBytes;
    if (toff + voff < a.strip_len)
      run_tile<K>(a.prog, voff, tab_lo, tab_hi, a.n_in, (uint32_t)a.strip_len, toff, SLOT_ARGS);
  }
}

// ---- batched execution: one persistent launch over many stripes
// Waves take (stripe, tile) work items from a device counter; each item runs
// its stripe's program on one tile.  Items and descriptors are read-only for
// the launch and are read through the scalar cache.
typedef const __attribute__((address_space(4))) StripeDesc *ConstDescPtr;
typedef const __attribute__((address_space(4))) uint32_t *ConstU32Ptr;

__global__ void batch_reset_kernel(uint32_t *counter) { *counter = 0u; }

template <int K>
__global__ void __launch_bounds__(256) slp_batch_kernel(BatchArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t voff = lane * 16u;
  v4u acc;
  v32u g0, g1, g2, g3, g4, g5;
  EC_SLOT_INIT(K);
  for (;;) {
    uint32_t it = 0;
    if (lane == 0) it = atomicAdd(a.counter, 1u);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= a.n_items) break;
    const uint32_t stripe = ((ConstU32Ptr)(uintptr_t)a.items)[2 * it];
    const uint32_t tile = ((ConstU32Ptr)(uintptr_t)a.items)[2 * it + 1];
    ConstDescPtr d = (ConstDescPtr)(uintptr_t)(a.stripes + stripe);
    const uint32_t *prog = d->prog;
    const uint32_t n_in = d->n_in, strip_len = d->strip_len;
    // lane b holds the pointer of block b of this stripe
    const uint64_t p = lane < (uint32_t)kMaxBlocks ? a.stripes[stripe].blk[lane] : 0ull;
    const uint32_t tab_lo = (uint32_t)p, tab_hi = (uint32_t)(p >> 32);
    for (uint32_t t = 0; t < a.tiles_per_item; ++t) {
      const uint64_t toff = (uint64_t)(tile + t) * kTileBytes;
      if (toff >= strip_len) break;
      if (toff + voff < strip_len) run_tile<K>(prog, voff, tab_lo, tab_hi, n_in, strip_len, toff, SLOT_ARGS);
    }
  }
}

int batch_launch(int slots, const BatchArgs &a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, stream, a.counter);
  switch (slots) {
    case 16: hipLaunchKernelGGL(slp_batch_kernel<16>, dim3(grid), dim3(256), 0, stream, a); break;
    case 24: hipLaunchKernelGGL(slp_batch_kernel<24>, dim3(grid), dim3(256), 0, stream, a); break;
    case 32: hipLaunchKernelGGL(slp_batch_kernel<32>, dim3(grid), dim3(256), 0, stream, a); break;
    case 40: hipLaunchKernelGGL(slp_batch_kernel<40>, dim3(grid), dim3(256), 0, stream, a); break;
    case 48: hipLaunchKernelGGL(slp_batch_kernel<48>, dim3(grid), dim3(256), 0, stream, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Plain device copy (16 B per lane, grid-stride): the bandwidth ceiling the
// executor is compared with, and the calibration kernel for byte counters.
__global__ void __launch_bounds__(256) copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                   uint64_t n16) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * 256u)
    dst[i] = src[i];
}

int copy_launch(const void *src, void *dst, uint64_t bytes, hipStream_t stream) {
  const uint64_t n16 = bytes / 16;
  const int grid = (int)std::min<uint64_t>((n16 + 255) / 256, 256u * 64u);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, (const uint4 *)src, (uint4 *)dst, n16);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int exec_launch(int slots, const ExecArgs &a, int grid, hipStream_t stream) {
  switch (slots) {
    case 16: hipLaunchKernelGGL(slp_exec_kernel<16>, dim3(grid), dim3(256), 0, stream, a); break;
    case 24: hipLaunchKernelGGL(slp_exec_kernel<24>, dim3(grid), dim3(256), 0, stream, a); break;
    case 32: hipLaunchKernelGGL(slp_exec_kernel<32>, dim3(grid), dim3(256), 0, stream, a); break;
    case 40: hipLaunchKernelGGL(slp_exec_kernel<40>, dim3(grid), dim3(256), 0, stream, a); break;
    case 48: hipLaunchKernelGGL(slp_exec_kernel<48>, dim3(grid), dim3(256), 0, stream, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace ec
