// ceiling.hip -- the bandwidth references the executor is measured against.
//
//  * copy_kernel: a plain device copy, the best of the variants measured on
//    the chip (non-temporal 16-byte loads and stores, two per lane per step,
//    16 workgroups of 256 lanes per compute unit, grid-stride): 0.78 of the
//    8 TB/s peak on 448 MiB, against 0.64 for one plain load and store per
//    lane on a large grid.  Also the calibration kernel for byte counters.
//  * stream_kernel: one launch of the executor's data movement with no
//    program: every tile reads all input strip-tiles and writes all output
//    strip-tiles (1 KiB of each per wave, non-temporal, the same tile order),
//    each output the XOR of the tile's inputs.  It is the ceiling for the
//    coding launch's access pattern, which reads many strips at one offset
//    and writes the outputs after the last read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "exec.hpp"
#include "tile_order.hpp"

namespace ec {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4u load_nt(const void *p) { return __builtin_nontemporal_load((const v4u *)p); }
__device__ __forceinline__ void store_nt(void *p, v4u v) { __builtin_nontemporal_store(v, (v4u *)p); }

// Accesses at a block address held as an integer, in the global address
// space: a pointer made from an integer is generic, and generic (flat)
// loads here were each followed by a wait for all of them.
typedef __attribute__((address_space(1))) const v4u global_cv4u;
typedef __attribute__((address_space(1))) v4u global_v4u;
__device__ __forceinline__ v4u load_nt_at(uint64_t base, uint64_t off) {
  return __builtin_nontemporal_load((global_cv4u *)(base + off));
}
__device__ __forceinline__ void store_nt_at(uint64_t base, uint64_t off, v4u v) {
  __builtin_nontemporal_store(v, (global_v4u *)(base + off));
}

constexpr int kCopyUnroll = 2;        // 16-byte elements per lane per step
constexpr int kCopyGroupsPerCu = 16;  // workgroups of 256 lanes per compute unit

__global__ void __launch_bounds__(256) copy_kernel(const v4u *__restrict__ src, v4u *__restrict__ dst, uint64_t n16) {
  const uint64_t step = (uint64_t)gridDim.x * 256 * kCopyUnroll;
  for (uint64_t base = (uint64_t)blockIdx.x * 256 * kCopyUnroll; base < n16; base += step) {
    v4u v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const uint64_t i = base + u * 256 + threadIdx.x;
      if (i < n16) v[u] = load_nt(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const uint64_t i = base + u * 256 + threadIdx.x;
      if (i < n16) store_nt(dst + i, v[u]);
    }
  }
}

int copy_launch(const void *src, void *dst, uint64_t bytes, int n_cus, hipStream_t stream) {
  const uint64_t n16 = bytes / 16;
  const uint64_t per_group = 256ull * kCopyUnroll;
  const int grid = (int)std::max<uint64_t>(
      1, std::min<uint64_t>((n16 + per_group - 1) / per_group, (uint64_t)n_cus * kCopyGroupsPerCu));
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, (const v4u *)src, (v4u *)dst, n16);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void __launch_bounds__(256) stream_kernel(ExecArgs a, uint32_t n_out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t n_waves = gridDim.x * 4u;
  const uint64_t sl = a.strip_len;
  for (uint32_t k = wave; k < a.n_tiles; k += n_waves) {
    const uint64_t off = (uint64_t)tile_of(k, a.seg_shift, a.seg_mask, a.seg_tiles) * kTileBytes + lane * 16u;
    if (off >= sl) continue;  // lanes past the end of a ragged last tile
    v4u acc = {0u, 0u, 0u, 0u};
    for (uint32_t i = 0; i < a.n_in; ++i) {
      v4u v[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = load_nt_at(a.blk[i], c * sl + off);
#pragma unroll
      for (int c = 0; c < 8; ++c) acc ^= v[c];
    }
    for (uint32_t j = 0; j < n_out; ++j) {
#pragma unroll
      for (int c = 0; c < 8; ++c) store_nt_at(a.blk[a.n_in + j], c * sl + off, acc);
    }
  }
}

int stream_launch(const ExecArgs &a, uint32_t n_out, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(stream_kernel, dim3(grid), dim3(256), 0, stream, a, n_out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ec
