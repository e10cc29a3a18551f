// native.hpp -- straight-line gfx950 kernels of compiled programs.
//
// A program's records (bytecode.hpp) are a fixed sequence of strip loads,
// register XORs and strip stores per tile.  native_source() writes them out
// as one inline-asm block of plain gfx950 instructions with every register
// slot a fixed VGPR group, so a tile runs with no record dispatch, register
// indexing or record-window loads: the interpreter's work without the
// interpreter.  The source is compiled at run time with hiprtc (host only,
// no device needed) and loaded per device on first use.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ec.h"

namespace ec {

// Arguments of a native kernel; the generated source declares the same
// layout.  blk: the input blocks, then the output blocks; strips of sl
// bytes; the tile order of tile_order.hpp.
struct NativeArgs {
  uint64_t blk[32];
  uint32_t sl, n_tiles, seg_shift, seg_mask, seg_tiles;
  uint32_t n_parts;  // work item k: part k % n_parts of tile k / n_parts
};

// Native kernels a program can have: the whole program, its pair parts
// and its block parts (EC_NATIVE_WHOLE, EC_NATIVE_PAIRS, EC_NATIVE_BLOCKS:
// kernel k for bit 1 << k).
constexpr int kNativeKernels = 3;

// Name of the kernel in every generated source.
constexpr const char *kNativeKernel = "ec_native_kernel";

// The source of the native kernel for `parts`, the records of one program
// or of the parts of a row split (records for `slots` register slots,
// reading and writing n_blocks blocks): with several parts, work item k
// runs part k % n_parts on tile k / n_parts, as the interpreter's split
// launches do.  Strip loads and stores are non-temporal, as the
// interpreter's.
std::string native_source(const std::vector<std::vector<uint32_t>> &parts, int slots, int n_blocks);

// Compiles `src` for gfx950; the code object in *code.  EC_ERR_UNSUPPORTED
// with the compiler's log in *log when it fails.
ec_status native_compile(const std::string &src, std::vector<char> *code, std::string *log);

// The kernel of `code` on device `dev` (the current device): loaded once
// per device and code object, kept until the process ends.  *per_cu: the
// workgroups of 256 lanes a compute unit holds at once.
ec_status native_function(int dev, const std::vector<char> &code, hipFunction_t *fn, int *per_cu);

// Launches `fn` on `grid` workgroups of 256 lanes; 0 on success.
int native_launch(hipFunction_t fn, const NativeArgs &a, int grid, hipStream_t stream);

}  // namespace ec
