#!/usr/bin/env python3
"""Writes exec.hip, the gfx950 executor, and staged.hip, its variant that
stages each tile in LDS, from the tables below.

Run from this directory after changing it:  python3 gen_exec.py
The record format it interprets is described in bytecode.hpp.
"""
import os

SLOT_BUDGETS = (24, 32, 36, 38, 40, 44, 48, 56, 60)
WA, WB = 36, 52          # the two 16-SGPR record windows
MAX_OPS = 14
STEP_BYTES = 20
MAX_WAIT = 63


def groups(K):
    """Pinned VGPR groups covering the K slots (v[4 : 4+4K)): 32-register
    groups, then a 16 and an 8 if needed."""
    out, lo, left = [], 4, 4 * K
    for size in (32, 16, 8):
        while left >= size:
            out.append((lo, size))
            lo += size
            left -= size
    assert left == 0, K
    return out


def vtype(size):
    return {32: "v32u", 16: "v16u", 8: "v8u"}[size]


def operands(K, mode):
    """Asm operand list for the accumulator and the slot groups."""
    c = {"inout": "+", "out": "="}[mode]
    ops = ['"%s{v[0:3]}"(acc)' % c]
    for i, (lo, size) in enumerate(groups(K)):
        ops.append('"%s{v[%d:%d]}"(g%d)' % (c, lo, lo + size - 1, i))
    # the prefetch target: written by loads that may still be in flight when
    # an asm statement ends, so pinned like the slots and never used
    ops.append('"%s{v%d}"(junk)' % (c, 4 + 4 * K))
    return ", ".join(ops)


def decls(K):
    return "v4u acc;\n  uint32_t junk;\n  " + " ".join("%s g%d;" % (vtype(size), i)
                                                      for i, (lo, size) in enumerate(groups(K)))


def asm_lines(lines):
    return "\n".join('      "%s\\n\\t"' % l for l in lines)


CLOBBERS = ", ".join('"s%d"' % r for r in range(36, 96)) + ', "scc"'


def handler(K, kind, W, O, run_base, h_other, lds=False):
    """One record handler for window W (the next record is loaded into O).
    lds: strips are read from the workgroup's staged copy of the tile in LDS
    (ds_read_b128) instead of from global memory."""
    nxt = ["s_bfe_u32 s74, s%d, 0x7000c" % W,           # record bytes
           "s_add_u32 s68, s68, s74",
           "s_load_dwordx16 s[%d:%d], %%[prog], s68" % (O, O + 15)]
    wait = ["s_and_b32 s74, s%d, 0x1f8" % (W + 1),     # 8 * wait
            "s_add_u32 s80, s94, s74",
            "s_addc_u32 s81, s95, 0",
            "s_swappc_b64 s[78:79], s[80:81]"]
    pull = ["s_and_b32 s74, s%d, 0xff" % W,            # 4 * pull slot
            "s_set_gpr_idx_on s74, gpr_idx(SRC0)",
            "v_mov_b32_e32 v0, v4", "v_mov_b32_e32 v1, v5",
            "v_mov_b32_e32 v2, v6", "v_mov_b32_e32 v3, v7",
            "s_set_gpr_idx_off"]
    addr = ["s_bfe_u32 s74, s%d, 0x50013" % (W + 1),   # block
            "v_readlane_b32 s72, %[tlo], s74",
            "v_readlane_b32 s73, %[thi], s74",
            "s_bfe_u32 s75, s%d, 0x30018" % (W + 1),   # strip of the block
            "s_mul_i32 s75, s75, %[sl]",
            "s_add_u32 s72, s72, s75",
            "s_addc_u32 s73, s73, 0",
            # five wait states between the v_readlane SGPR writes and the
            # memory instruction reading the address
            "s_nop 4"]
    ld = ["s_bfe_u32 s74, s%d, 0xa0009" % (W + 1),     # 16 * ld slot
          # (the host validates every field; the clamps keep a computed jump
          # inside its table whatever the word holds)
          "s_min_u32 s74, s74, %d" % (16 * (K - 1)),
          "s_add_u32 s80, s92, s74",
          "s_addc_u32 s81, s93, 0",
          "s_swappc_b64 s[78:79], s[80:81]"]
    # strips are streamed once: loads and stores are non-temporal (measured:
    # 0.58 -> 0.69 of peak HBM bandwidth on the 64 MiB-block encode).
    # Device-scope (sc1) or plain stores are slower here (64 MiB encode
    # 0.168 and 0.165 against 0.163 ms; a batch of 1 MiB decodes 4.05
    # against 3.49 ms).  They look faster only when a launch rewrites the
    # lines the launch before it wrote, which the memory-side cache then
    # absorbs; with outputs that change every launch they are no faster.
    store = ["global_store_dwordx4 %[voff], v[0:3], s[72:73] nt",
             # one wait state before a VALU may overwrite the store's data
             "s_nop 1"]
    run = ["s_bfe_u32 s74, s%d, 0x90013" % W,          # run entry offset
           "s_min_u32 s74, s74, %d" % (MAX_OPS * STEP_BYTES),
           "s_add_u32 s80, s%d, s74" % run_base,
           "s_addc_u32 s81, s%d, 0" % (run_base + 1),
           "s_setpc_b64 s[80:81]"]
    # staged: strip (block b, strip c) of the tile sits at LDS byte
    # lbase + (8 b + c) * 1 KiB, lane l's 16 bytes at + 16 l; the address
    # goes through the spare register (no prefetch records run here)
    laddr = ["s_bfe_u32 s74, s%d, 0x50013" % (W + 1),  # block
             "s_bfe_u32 s75, s%d, 0x30018" % (W + 1),  # strip of the block
             "s_lshl3_add_u32 s74, s74, s75",
             "s_lshl_b32 s74, s74, 10",
             "s_add_u32 s74, s74, %[lbase]",
             "v_add_u32_e32 v%d, s74, %%[voff]" % (4 + 4 * K)]
    if lds:
        # an LDS read completes within its record (the window's wait for
        # lgkmcnt(0) also covers it), so the wait records have nothing to do
        # and the prefetch records are skipped
        body = {
            0: nxt + run,
            1: nxt + pull + run,
            2: nxt + pull + laddr + ld + run,
            3: nxt + pull + run,
            4: nxt + pull + addr + store + run,
            5: nxt + laddr + ld + run,
            6: ["s_branch 99f"],
            7: nxt + run,
        }[kind]
        return [".p2align 9"] + body
    body = {
        0: nxt + run,
        1: nxt + wait + pull + run,
        2: nxt + wait + pull + addr + ld + run,
        3: nxt + pull + run,
        4: nxt + pull + addr + store + run,
        5: nxt + addr + ld + run,
        6: ["s_branch 99f"],
        7: nxt + addr + ["global_load_dword v%d, %%[voff], s[72:73]" % (4 + 4 * K)] + run,
    }[kind]
    return [".p2align 9"] + body


def run_table(W, O, h_other):
    lines = []
    for i in range(MAX_OPS):
        lines += ["s_set_gpr_idx_on s%d, gpr_idx(SRC0,DST)" % (W + 15 - i),
                  "v_xor_b32_e32 v4, v4, v0", "v_xor_b32_e32 v5, v5, v1",
                  "v_xor_b32_e32 v6, v6, v2", "v_xor_b32_e32 v7, v7, v3"]
    lines += ["s_set_gpr_idx_off",
              "s_waitcnt lgkmcnt(0)",                 # the next record's window
              "s_and_b32 s74, s%d, 0xe00" % O,        # its kind * 512
              "s_add_u32 s80, s%d, s74" % h_other,
              "s_addc_u32 s81, s%d, 0" % (h_other + 1),
              "s_setpc_b64 s[80:81]"]
    return lines


def program_asm(K, lds=False):
    L = ["s_mov_b32 s68, 0",
         "s_load_dwordx16 s[%d:%d], %%[prog], 0x0" % (WA, WA + 15),
         "s_getpc_b64 s[82:83]",
         "90:"]
    for reg, label in ((84, 91), (86, 92), (88, 93), (90, 94), (92, 95), (94, 96)):
        L += ["s_add_u32 s%d, s82, %df-90b" % (reg, label), "s_addc_u32 s%d, s83, 0" % (reg + 1)]
    L += ["s_waitcnt lgkmcnt(0)",
          "s_and_b32 s74, s%d, 0xe00" % WA,
          "s_add_u32 s80, s84, s74",
          "s_addc_u32 s81, s85, 0",
          "s_setpc_b64 s[80:81]"]
    for W, O, run_base, h_other, label in ((WA, WB, 88, 86, 91), (WB, WA, 90, 84, 92)):
        for kind in range(8):
            h = handler(K, kind, W, O, run_base, h_other, lds)
            if kind == 0:
                h = h[:1] + ["%d:" % label] + h[1:]
            L += h
    L += [".p2align 2", "93:"] + run_table(WA, WB, 86)
    L += ["94:"] + run_table(WB, WA, 84)
    L += ["95:"]
    for k in range(K):
        if lds:  # 8 + 4 + 4 bytes, like the global entry
            L += ["ds_read_b128 v[%d:%d], v%d" % (4 + 4 * k, 7 + 4 * k, 4 + 4 * K),
                  "s_setpc_b64 s[78:79]", "s_nop 0"]
        else:
            L += ["global_load_dwordx4 v[%d:%d], %%[voff], s[72:73] nt" % (4 + 4 * k, 7 + 4 * k),
                  "s_setpc_b64 s[78:79]", "s_nop 0"]
    L += ["96:"]
    for k in range(MAX_WAIT + 1):
        L += ["s_waitcnt vmcnt(%d)" % k, "s_setpc_b64 s[78:79]"]
    L += ["99:"]
    return L


INTRO = r'''// exec.hip -- gfx950 executor for push-form XOR programs.
// GENERATED by gen_exec.py -- edit that file and regenerate.
//
// One wave runs the whole program, or one row-split part of it, on one tile:
// 64 lanes x 16 bytes = 1 KiB of every input and output strip (the blocked
// loop of Sec. 6.1; the tile is the paper's block size).  The accumulator is pinned to v[0:3] and K
// register slots of 16 bytes per lane to v[4 : 4+4K).  The program is a
// stream of records (bytecode.hpp) read through the scalar cache, two
// 16-word windows in turn, the next record's window loading while the
// current record runs.  The interpreter is one asm block:
//  * dispatch: the record's kind * 512 is the byte offset of its handler
//    (handlers are 512-byte aligned), so a record costs one computed jump;
//  * pull: acc = slot[i] through s_set_gpr_idx_on (VGPR indexing);
//  * run: a computed jump into 14 unrolled 20-byte steps, each an indexed
//    slot ^= acc (four v_xor_b32), entered so that exactly the record's
//    operands execute; the run falls through into the next dispatch;
//  * strip loads land in their slot through a table of K global_load_dwordx4
//    (16 B per lane, 1 KiB per wave, coalesced, non-temporal: every strip
//    is streamed once), stores write acc; vmcnt waits are the host's exact
//    counts, through a 64-entry table.
// Temporaries never leave the registers (the deforestation of Sec. 5); the
// host validates every record before the program reaches the device.
'''

DEFS = r'''#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bytecode.hpp"
#include "exec.hpp"
#include "tile_order.hpp"

namespace ec {

typedef uint32_t v32u __attribute__((ext_vector_type(32)));
typedef uint32_t v16u __attribute__((ext_vector_type(16)));
typedef uint32_t v8u __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

static_assert(bc::kMaxOps == %(MAX_OPS)d && bc::kRunStepBytes == %(STEP)d && bc::kMaxWait == %(MAXW)d,
              "record format and executor tables disagree");

// Lane b of the result: block b's pointer plus the tile offset.  The
// executor reads it from any lane with v_readlane, also in a ragged last
// tile where only the lanes below the strip's end are active, so it must be
// computed with every lane on: a volatile asm statement is never moved into
// the partial-tile branch.
__device__ __forceinline__ uint64_t tile_table(uint64_t tab, uint64_t toff) {
  uint64_t t;
  asm volatile("v_lshl_add_u64 %%0, %%1, 0, %%2" : "=v"(t) : "s"(toff), "v"(tab));
  return t;
}

typedef const __attribute__((address_space(4))) StripeDesc *ConstDescPtr;
typedef const __attribute__((address_space(4))) uint32_t *ConstU32Ptr;

'''

HEAD = INTRO + DEFS


PER_K = r'''// ---- %(K)d slots
#define EC_INIT_%(K)d asm volatile(%(INIT)s : %(OUT)s)
#define EC_RUN_%(K)d(prog_, voff_, tlo_, thi_, sl_)  \
  asm volatile(                                  \
%(PROGRAM)s
      : %(INOUT)s                                \
      : [prog] "s"(prog_), [voff] "v"(voff_), [tlo] "v"(tlo_), [thi] "v"(thi_), [sl] "s"(sl_) \
      : %(CLOB)s)

__global__ void __launch_bounds__(256) slp_exec_kernel_%(K)d(ExecArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  // wave index as a scalar: every per-tile address below is wave-uniform
  const uint32_t wave = blockIdx.x * 4u + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t n_waves = gridDim.x * 4u;
  // lane b holds the pointer of block b
  uint64_t tab = lane < (uint32_t)kMaxBlocks ? a.blk[lane] : 0ull;
  // wait for the table here, once: the compiler cannot see the executor's
  // own memory operations and would otherwise wait for them at every tile
  asm volatile("s_waitcnt vmcnt(0)" : "+v"(tab));
  const uint32_t voff = lane * 16u;
  const uint32_t sl = (uint32_t)a.strip_len;
  const uint32_t *prog = a.prog;
  %(DECLS)s
  EC_INIT_%(K)d;
  // work item k: part k %% n_parts of tile k / n_parts (the whole program
  // on tile k when n_parts = 1)
  const uint32_t n_parts = a.n_parts;
  const uint32_t n_work = a.n_tiles * n_parts;
  for (uint32_t k = wave; k < n_work; k += n_waves) {
    uint32_t kt = k;
    const uint32_t *pk = prog;
    if (n_parts > 1) {
      kt = k / n_parts;
      pk = prog + a.part_off[k - kt * n_parts];
    }
    const uint32_t tile = tile_of(kt, a.seg_shift, a.seg_mask, a.seg_tiles);
    const uint64_t toff = (uint64_t)tile * kTileBytes;
    const uint64_t t = tile_table(tab, toff);
    const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
    if (toff + voff < sl) EC_RUN_%(K)d(pk, voff, tlo, thi, sl);
  }
}

// Workgroups take work items from a device counter, 4 `chunk`s of
// consecutive items per atomic add, and wave w of the workgroup runs chunk
// w: the host lists a stripe's tiles consecutively, so the 4 waves of a
// compute unit run neighbouring tiles side by side, and a cache line that
// two neighbouring tiles share (a strip that starts off a 128-byte line)
// is fetched once into that unit's L2 rather than by two units.  Every
// wave leaves the loop on the same shared value, so each reaches every
// barrier.  An item covers tiles_per_item tiles of its stripe.  Items,
// descriptors and block tables are read through the scalar cache; the
// block table is rebuilt only when the stripe changes.
__global__ void __launch_bounds__(256) slp_batch_kernel_%(K)d(BatchArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t voff = lane * 16u;
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  __shared__ uint32_t group_first;
  %(DECLS)s
  EC_INIT_%(K)d;
  uint32_t cur = 0xffffffffu, tab_lo = 0, tab_hi = 0;
  for (;;) {
    if (threadIdx.x == 0) group_first = atomicAdd(a.counter, 4u * a.chunk);
    __syncthreads();
    const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)group_first);
    __syncthreads();  // every wave has read it before the next add writes it
    if (base >= a.n_items) break;
    const uint32_t first = base + wave * a.chunk;
    const uint32_t last = min(first + a.chunk, a.n_items);
    for (uint32_t it = first; it < last; ++it) {
      const uint32_t stripe = ((ConstU32Ptr)(uintptr_t)a.items)[2 * it];
      const uint32_t word = ((ConstU32Ptr)(uintptr_t)a.items)[2 * it + 1];
      const uint32_t tile = word & kItemTileMask, part = word >> kItemPartShift;
      ConstDescPtr d = (ConstDescPtr)(uintptr_t)(a.stripes + stripe);
      const uint32_t *prog = d->prog + d->part_off[part];
      const uint32_t sl = d->strip_len;
      if (stripe != cur) {
        // lane b <- pointer of block b, written lane by lane from scalar
        // loads (all 32 entries: the host zero-fills the unused ones)
%(WRITELANES)s
        cur = stripe;
      }
      const uint64_t tab = ((uint64_t)tab_hi << 32) | tab_lo;
      for (uint32_t k = 0; k < a.tiles_per_item; ++k) {
        const uint64_t toff = (uint64_t)(tile + k) * kTileBytes;
        if (toff >= sl) break;
        const uint64_t t = tile_table(tab, toff);
        const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
        if (toff + voff < sl) EC_RUN_%(K)d(prog, voff, tlo, thi, sl);
      }
    }
  }
}

'''

TAIL = r'''__global__ void batch_reset_kernel(uint32_t *counter) { *counter = 0u; }

int exec_launch(int slots, const ExecArgs &a, int grid, hipStream_t stream) {
  switch (slots) {
%(EXEC_CASES)s
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int batch_launch(int slots, const BatchArgs &a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, stream, a.counter);
  switch (slots) {
%(BATCH_CASES)s
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace ec
'''


STAGED_INTRO = r'''// staged.hip -- gfx950 executor with each tile staged in LDS.
// GENERATED by gen_exec.py -- edit that file and regenerate.
//
// The 4 waves of a workgroup share one tile (1 KiB of every strip): they
// copy its input strip-tiles from global memory into LDS with LDS-DMA loads
// (global_load_lds_dwordx4: 16 B per lane, non-temporal), meet at a
// barrier, and each runs one part of the program, a quarter of the output
// rows, through the interpreter of exec.hip, whose strip loads here read the
// staged copy (ds_read_b128) instead of global memory; outputs are stored
// from the registers as there.  A second barrier ends the tile before the
// next one is staged.  Every input strip-tile leaves HBM once per tile
// whatever the number of parts, and a part's register slots hold only its
// own rows and temporaries: LDS is one more level between the registers and
// HBM (the multi-level hierarchy of Sec. 8), with the workgroups that share
// a compute unit overlapping one's staging with another's compute.
'''

PER_K_STAGED = r'''// ---- %(K)d slots
#define EC_INIT_%(K)d asm volatile(%(INIT)s : %(OUT)s)
#define EC_SRUN_%(K)d(prog_, voff_, tlo_, thi_, sl_, lbase_)  \
  asm volatile(                                  \
%(PROGRAM)s
      : %(INOUT)s                                \
      : [prog] "s"(prog_), [voff] "v"(voff_), [tlo] "v"(tlo_), [thi] "v"(thi_), [sl] "s"(sl_), \
        [lbase] "s"(lbase_)                      \
      : %(CLOB)s, "m0", "memory")

__global__ void __launch_bounds__(256) slp_staged_kernel_%(K)d(ExecArgs a) {
  extern __shared__ v4u stage[];  // 8 strip-tiles of 1 KiB per input block
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint64_t tab = lane < (uint32_t)kMaxBlocks ? a.blk[lane] : 0ull;
  asm volatile("s_waitcnt vmcnt(0)" : "+v"(tab));
  const uint32_t voff = lane * 16u;
  const uint32_t sl = (uint32_t)a.strip_len;
  const uint32_t n_strips = a.n_in * 8u;
  // wave w runs part w; waves beyond the parts only stage
  const bool runs = wave < a.n_parts;
  const uint32_t *pk = a.prog + a.part_off[runs ? wave : 0u];
  const uint32_t lbase = (uint32_t)(uintptr_t)stage;
  %(DECLS)s
  EC_INIT_%(K)d;
  for (uint32_t kt = blockIdx.x; kt < a.n_tiles; kt += gridDim.x) {
    const uint32_t tile = tile_of(kt, a.seg_shift, a.seg_mask, a.seg_tiles);
    const uint64_t toff = (uint64_t)tile * kTileBytes;
    const uint64_t t = tile_table(tab, toff);
    const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
    if (toff + voff < sl) {
      // strip-tile s = 8 b + c (block b, strip c) goes to stage[64 s ..]
      for (uint32_t s = wave; s < n_strips; s += 4u) {
        const uint32_t b = s >> 3;
        const uint64_t base = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)thi, (int)b) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)tlo, (int)b);
        const uint64_t src = base + (uint64_t)(s & 7u) * sl + voff;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(uintptr_t)src,
                                         (__attribute__((address_space(3))) void *)(stage + 64u * s), 16, 0,
                                         kStageNonTemporal);
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (runs && toff + voff < sl) EC_SRUN_%(K)d(pk, voff, tlo, thi, sl, lbase);
    __syncthreads();
  }
}

'''

STAGED_TAIL = r'''int staged_launch(int slots, const ExecArgs &a, int grid, uint32_t lds_bytes, hipStream_t stream) {
  switch (slots) {
%(CASES)s
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace ec
'''


def writelanes():
    """Lane b of (tab_lo, tab_hi) <- block b's pointer (v_writelane with an
    immediate lane: no per-lane compare masks)."""
    out = []
    for b in range(32):
        out.append('        { const uint64_t ptr = d->blk[%d];\n'
                   '          asm("v_writelane_b32 %%0, %%1, %d" : "+v"(tab_lo) : "s"((uint32_t)ptr));\n'
                   '          asm("v_writelane_b32 %%0, %%1, %d" : "+v"(tab_hi) : "s"((uint32_t)(ptr >> 32))); }'
                   % (b, b, b))
    return "\n".join(out)


def init_asm(K):
    regs = ["v_mov_b32_e32 v%d, 0" % r for r in range(4 + 4 * K + 1)]
    return '"' + "\\n\\t".join(regs) + '"'


def main(out_dir=None):
    """Writes exec.hip and staged.hip into out_dir (default: beside this
    file)."""
    out = HEAD % {"MAX_OPS": MAX_OPS, "STEP": STEP_BYTES, "MAXW": MAX_WAIT}
    for K in SLOT_BUDGETS:
        prog = "\n".join('      "%s\\n\\t"                     \\' % l for l in program_asm(K))
        out += PER_K % {"K": K, "INIT": init_asm(K), "OUT": operands(K, "out"), "INOUT": operands(K, "inout"),
                        "PROGRAM": prog, "CLOB": CLOBBERS, "DECLS": decls(K), "WRITELANES": writelanes()}
    exec_cases = "\n".join(
        "    case %d: hipLaunchKernelGGL(slp_exec_kernel_%d, dim3(grid), dim3(256), 0, stream, a); break;" % (K, K)
        for K in SLOT_BUDGETS)
    batch_cases = "\n".join(
        "    case %d: hipLaunchKernelGGL(slp_batch_kernel_%d, dim3(grid), dim3(256), 0, stream, a); break;" % (K, K)
        for K in SLOT_BUDGETS)
    out += TAIL % {"EXEC_CASES": exec_cases, "BATCH_CASES": batch_cases}
    here = out_dir or os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "exec.hip"), "w") as f:
        f.write(out)

    staged_defs = DEFS.replace('#include "exec.hpp"\n', '#include "exec.hpp"\n#include "staged.hpp"\n')
    staged = STAGED_INTRO + staged_defs % {"MAX_OPS": MAX_OPS, "STEP": STEP_BYTES, "MAXW": MAX_WAIT}
    staged += "// cache policy of the staging loads: non-temporal (each strip-tile is read once)\n"
    staged += "constexpr int kStageNonTemporal = 2;\n\n"
    for K in SLOT_BUDGETS:
        prog = "\n".join('      "%s\\n\\t"                     \\' % l for l in program_asm(K, lds=True))
        staged += PER_K_STAGED % {"K": K, "INIT": init_asm(K), "OUT": operands(K, "out"),
                                  "INOUT": operands(K, "inout"), "PROGRAM": prog, "CLOB": CLOBBERS,
                                  "DECLS": decls(K)}
    cases = "\n".join(
        "    case %d: hipLaunchKernelGGL(slp_staged_kernel_%d, dim3(grid), dim3(256), lds_bytes, stream, a); break;"
        % (K, K) for K in SLOT_BUDGETS)
    staged += STAGED_TAIL % {"CASES": cases}
    with open(os.path.join(here, "staged.hip"), "w") as f:
        f.write(staged)


if __name__ == "__main__":
    main()
