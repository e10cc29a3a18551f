// batch.cpp -- many stripes in one persistent launch.
//
// A batch is a table of stripe descriptors and a list of work items
// (stripe, first tile), uploaded once.  A launch resets the work counter with
// a one-thread kernel and starts the persistent executor, whose waves take
// chunks of items from the counter until the list is exhausted; both
// launches are captured into a HIP graph at build time, so a launch is one
// graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <utility>
#include <vector>

#include "../../include/ec.h"
#include "batch.hpp"
#include "exec.hpp"
#include "program.hpp"

using namespace ec;

struct ec_batch {
  int device = 0;
  int n_cus = 0;  // compute units of the device (read once: the query is slow)
  int slots = 0;
  int grid = 0;
  size_t n_items = 0, in_bytes = 0, out_bytes = 0;
  // device tables and their pinned host staging, grown on demand, never
  // shrunk (so refilling a batch in a serving loop allocates nothing)
  StripeDesc *d_desc = nullptr, *h_desc = nullptr;
  uint32_t *d_items = nullptr, *h_items = nullptr;
  uint32_t *d_counter = nullptr;
  size_t cap_desc = 0, cap_items = 0;
  std::vector<ByteRange> reads, writes;  // overlap-check workspaces, reused
  BatchArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~ec_batch() {
    int cur = 0;
    const bool swap = hipGetDevice(&cur) == hipSuccess && cur != device && hipSetDevice(device) == hipSuccess;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_desc) (void)hipFree(d_desc);
    if (d_items) (void)hipFree(d_items);
    if (d_counter) (void)hipFree(d_counter);
    if (h_desc) (void)hipHostFree(h_desc);
    if (h_items) (void)hipHostFree(h_items);
    if (swap) (void)hipSetDevice(cur);
  }
};

namespace {

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool by_first(const ByteRange &a, const ByteRange &b) {
  return a.first < b.first || (a.first == b.first && a.second < b.second);
}

// The stripes of one launch run in no defined order, so every byte written
// must be written by one output block only and read by none: the written
// ranges are pairwise disjoint and disjoint from every read range (reads
// may overlap each other).  Sorts both arrays and merges the reads in place.
bool disjoint_writes(ByteRange *reads, size_t n_reads, ByteRange *writes, size_t n_writes) {
  std::sort(writes, writes + n_writes, by_first);
  for (size_t k = 1; k < n_writes; ++k)
    if (writes[k].first < writes[k - 1].second) return false;
  std::sort(reads, reads + n_reads, by_first);
  size_t m = 0;  // merged read ranges, in reads[0, m)
  for (size_t k = 0; k < n_reads; ++k) {
    if (m && reads[k].first <= reads[m - 1].second)
      reads[m - 1].second = std::max(reads[m - 1].second, reads[k].second);
    else
      reads[m++] = reads[k];
  }
  for (size_t k = 0; k < n_writes; ++k) {
    const ByteRange &w = writes[k];
    // first merged read range ending after the write begins
    const ByteRange *it = std::upper_bound(reads, reads + m, w.first,
                                           [](uintptr_t x, const ByteRange &r) { return x < r.second; });
    if (it != reads + m && it->first < w.second) return false;
  }
  return true;
}

// The part offsets a stripe's work items name under the batch's split.
const std::vector<uint32_t> *split_offsets(const ec_program *prog, const BatchPlan &plan) {
  if (prog->split == EC_SPLIT_ROWS || (prog->split == EC_SPLIT_AUTO && plan.rows_fit))
    return prog->row_parts.empty() ? nullptr : &prog->row_part_off;
  if (prog->split == EC_SPLIT_PAIRS || (prog->split == EC_SPLIT_AUTO && plan.pairs_fit))
    return prog->pair_parts.empty() ? nullptr : &prog->pair_part_off;
  if (prog->split == EC_SPLIT_ALWAYS || (prog->split == EC_SPLIT_AUTO && plan.blocks_fit))
    return prog->parts.empty() ? nullptr : &prog->part_off;
  // a program that needs several passes over its inputs runs its pass parts
  if (prog->split == EC_SPLIT_PASSES || prog->split == EC_SPLIT_AUTO)
    return prog->pass_parts.empty() ? nullptr : &prog->pass_part_off;
  return nullptr;
}

uint32_t n_tiles_of(size_t block_bytes) { return (uint32_t)((block_bytes / 8 + kTileBytes - 1) / kTileBytes); }

}  // namespace

namespace ec {

ec_status batch_plan(const ec_stripe *stripes, int n_stripes, size_t tile_bytes, int n_cus, BatchPlan *plan) {
  if (!stripes || n_stripes <= 0 || !plan) return EC_ERR_ARG;
  if (tile_bytes == 0) tile_bytes = kTileBytes;
  if (tile_bytes % kTileBytes != 0 || tile_bytes / kTileBytes > 4096) return EC_ERR_UNSUPPORTED;
  BatchPlan pl;
  pl.tiles_per_item = (uint32_t)(tile_bytes / kTileBytes);
  uint64_t items_rows = 0, items_pairs = 0, items_blocks = 0;  // work items with each set of parts
  for (int s = 0; s < n_stripes; ++s) {
    const ec_stripe &st = stripes[s];
    const ec_program *prog = st.prog;
    if (!prog || !st.in || !st.out) return EC_ERR_ARG;
    if (st.block_bytes == 0 || st.block_bytes % 128 != 0) return EC_ERR_ALIGN;
    if (st.block_bytes / 8 > 0x1FFFFFFFull) return EC_ERR_UNSUPPORTED;
    if (s == 0) pl.slots = prog->slots;
    else if (prog->slots != pl.slots) return EC_ERR_UNSUPPORTED;  // one kernel instance per launch
    const int n_in = (int)prog->in_blocks.size(), n_out = (int)prog->out_blocks.size();
    for (int i = 0; i < n_in; ++i)
      if (!st.in[i]) return EC_ERR_ARG;
      else if (!aligned16(st.in[i])) return EC_ERR_ALIGN;
    for (int j = 0; j < n_out; ++j)
      if (!st.out[j]) return EC_ERR_ARG;
      else if (!aligned16(st.out[j])) return EC_ERR_ALIGN;
    const uint64_t n_tiles = n_tiles_of(st.block_bytes);
    items_rows += n_tiles * std::max<size_t>(1, prog->row_parts.size());
    items_pairs += n_tiles * std::max<size_t>(1, prog->pair_parts.size());
    items_blocks += n_tiles * std::max<size_t>(1, prog->parts.size());
    pl.in_bytes += (size_t)n_in * st.block_bytes;
    pl.out_bytes += (size_t)n_out * st.block_bytes;
    pl.n_ranges_in += (size_t)n_in;
    pl.n_ranges_out += (size_t)n_out;
  }
  // Row split as for one stripe, decided for the whole batch: row parts
  // when one wave per (tile, row part) of every stripe leaves at most two
  // waves per SIMD, else pair parts when theirs do, else block parts when
  // all theirs are resident, else none (stripes compiled with another
  // policy than EC_SPLIT_AUTO take their own choice).
  const uint64_t resident_waves = 4ull * (uint64_t)n_cus * waves_per_simd(pl.slots);
  const uint64_t fine_waves = 2ull * 4 * (uint64_t)n_cus;  // two waves per SIMD
  pl.rows_fit = items_rows <= fine_waves;
  pl.pairs_fit = !pl.rows_fit && items_pairs <= fine_waves;
  pl.blocks_fit = !pl.rows_fit && !pl.pairs_fit && items_blocks <= resident_waves;
  for (int s = 0; s < n_stripes; ++s) {
    const std::vector<uint32_t> *off = split_offsets(stripes[s].prog, pl);
    const uint64_t n_its = (n_tiles_of(stripes[s].block_bytes) + pl.tiles_per_item - 1) / pl.tiles_per_item;
    pl.n_items += n_its * (off ? off->size() : 1);
  }
  if (pl.n_items > 0xFFFFFFFFull) return EC_ERR_UNSUPPORTED;
  *plan = pl;
  return EC_OK;
}

ec_status batch_fill(const ec_stripe *stripes, int n_stripes, const BatchPlan &plan, int dev, bool upload,
                     StripeDesc *desc, uint32_t *items, ByteRange *reads, ByteRange *writes) {
  const bool check = reads && writes;
  size_t nr = 0, nw = 0, w = 0;
  for (int s = 0; s < n_stripes; ++s) {
    const ec_stripe &st = stripes[s];
    const ec_program *prog = st.prog;
    const int n_in = (int)prog->in_blocks.size(), n_out = (int)prog->out_blocks.size();
    StripeDesc &d = desc[s];
    std::memset(&d, 0, sizeof d);  // unused block entries are zero (the kernel reads all 32)
    for (int i = 0; i < n_in; ++i) {
      d.blk[i] = (uint64_t)(uintptr_t)st.in[i];
      if (check) reads[nr++] = {(uintptr_t)st.in[i], (uintptr_t)st.in[i] + st.block_bytes};
    }
    for (int j = 0; j < n_out; ++j) {
      d.blk[n_in + j] = (uint64_t)(uintptr_t)st.out[j];
      if (check) writes[nw++] = {(uintptr_t)st.out[j], (uintptr_t)st.out[j] + st.block_bytes};
    }
    ec_program *mp = const_cast<ec_program *>(prog);
    ec_status ws = EC_OK;
    d.prog = upload ? mp->device_words(dev, &ws) : mp->device_words_present(dev);
    if (!d.prog) return upload ? ws : EC_ERR_ARG;
    d.n_blocks = (uint32_t)(n_in + n_out);
    d.strip_len = (uint32_t)(st.block_bytes / 8);
    const std::vector<uint32_t> *off = split_offsets(prog, plan);
    const uint32_t n_parts = off ? (uint32_t)off->size() : 1u;
    for (uint32_t q = 0; q < (uint32_t)kMaxRowParts; ++q) d.part_off[q] = off && q < n_parts ? (*off)[q] : 0u;
    const uint32_t n_its = (n_tiles_of(st.block_bytes) + plan.tiles_per_item - 1) / plan.tiles_per_item;
    // Strips a multiple of 4 MiB apart: groups of 4 consecutive items on 4
    // neighbouring tiles, consecutive groups in 8 distant segments of the
    // strips (the single-stripe launch's tile order).
    const bool spread = d.strip_len % (4u << 20) == 0 && n_its % 32 == 0;
    for (uint32_t k = 0; k < n_its; ++k) {
      const uint32_t g = k / 4;
      const uint32_t i = spread ? (g & 7u) * (n_its >> 3) + (g >> 3) * 4 + k % 4 : k;
      for (uint32_t q = 0; q < n_parts; ++q) {  // a tile's parts side by side
        items[w++] = (uint32_t)s;
        items[w++] = i * plan.tiles_per_item | q << kItemPartShift;
      }
    }
  }
  if (check && !disjoint_writes(reads, nr, writes, nw)) return EC_ERR_ARG;
  return EC_OK;
}

int batch_grid(const BatchPlan &plan, int n_cus) {
  return (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)n_cus * waves_per_simd(plan.slots),
                                                      (plan.n_items + 3) / 4));
}

}  // namespace ec

namespace {

// Grows the device tables and their pinned staging to hold n_desc stripes
// and n_words item words (never shrinks).
ec_status grow(ec_batch *b, size_t n_desc, size_t n_words) {
  if (n_desc > b->cap_desc) {
    const size_t cap = std::max(n_desc, 2 * b->cap_desc);
    StripeDesc *d = nullptr, *h = nullptr;
    if (hipMalloc((void **)&d, cap * sizeof(StripeDesc)) != hipSuccess) return EC_ERR_NOMEM;
    if (hipHostMalloc((void **)&h, cap * sizeof(StripeDesc), hipHostMallocDefault) != hipSuccess) {
      (void)hipFree(d);
      return EC_ERR_NOMEM;
    }
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    b->d_desc = d;
    b->h_desc = h;
    b->cap_desc = cap;
  }
  if (n_words > b->cap_items) {
    const size_t cap = std::max(n_words, 2 * b->cap_items);
    uint32_t *d = nullptr, *h = nullptr;
    if (hipMalloc((void **)&d, cap * sizeof(uint32_t)) != hipSuccess) return EC_ERR_NOMEM;
    if (hipHostMalloc((void **)&h, cap * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
      (void)hipFree(d);
      return EC_ERR_NOMEM;
    }
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->h_items) (void)hipHostFree(b->h_items);
    b->d_items = d;
    b->h_items = h;
    b->cap_items = cap;
  }
  return EC_OK;
}

}  // namespace

namespace ec {

ec_status batch_set(ec_batch *b, const ec_stripe *stripes, int n_stripes, size_t tile_bytes, ec_stream stream,
                    bool check_overlap) {
  if (!b || !stripes || n_stripes <= 0) return EC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return EC_ERR_DEVICE;
  BatchPlan plan;
  ec_status st = batch_plan(stripes, n_stripes, tile_bytes, b->n_cus, &plan);
  if (st != EC_OK) return st;
  st = grow(b, (size_t)n_stripes, 2 * plan.n_items);
  if (st != EC_OK) return st;
  // Tables straight into the pinned staging (the previous launch of this
  // batch, and so its copies, must have completed).
  ByteRange *reads = nullptr, *writes = nullptr;
  if (check_overlap) {
    b->reads.resize(plan.n_ranges_in);
    b->writes.resize(plan.n_ranges_out);
    reads = b->reads.data();
    writes = b->writes.data();
  }
  st = batch_fill(stripes, n_stripes, plan, dev, true, b->h_desc, b->h_items, reads, writes);
  if (st != EC_OK) return st;
  const hipStream_t hs = (hipStream_t)stream;
  if (hipMemcpyAsync(b->d_desc, b->h_desc, (size_t)n_stripes * sizeof(StripeDesc), hipMemcpyHostToDevice, hs) !=
          hipSuccess ||
      hipMemcpyAsync(b->d_items, b->h_items, 2 * plan.n_items * sizeof(uint32_t), hipMemcpyHostToDevice, hs) !=
          hipSuccess)
    return EC_ERR_DEVICE;
  b->slots = plan.slots;
  b->n_items = plan.n_items;
  b->in_bytes = plan.in_bytes;
  b->out_bytes = plan.out_bytes;
  b->args.stripes = b->d_desc;
  b->args.items = b->d_items;
  b->args.n_items = (uint32_t)b->n_items;
  b->args.tiles_per_item = plan.tiles_per_item;
  b->grid = batch_grid(plan, b->n_cus);
  // One item per atomic add: waves running side by side then work on
  // neighbouring tiles, which the memory system rewards more than larger
  // chunks save on the adds (measured on the 8192-stripe mix: 12.2 ms with
  // 1 item, 13.2 with 2, 14.4 with 16).
  b->args.chunk = 1;
  b->args.counter = b->d_counter;
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return EC_OK;
}

}  // namespace ec

extern "C" {

ec_status ec_batch_create(ec_batch **out) {
  if (!out) return EC_ERR_ARG;
  *out = nullptr;
  std::unique_ptr<ec_batch> b(new (std::nothrow) ec_batch);
  if (!b) return EC_ERR_NOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) return EC_ERR_DEVICE;
  if (hipDeviceGetAttribute(&b->n_cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
    return EC_ERR_DEVICE;
  if (hipMalloc((void **)&b->d_counter, 256) != hipSuccess) return EC_ERR_NOMEM;
  *out = b.release();
  return EC_OK;
}

ec_status ec_batch_set(ec_batch *b, const ec_stripe *stripes, int n_stripes, size_t tile_bytes, ec_stream stream) {
  return batch_set(b, stripes, n_stripes, tile_bytes, stream, true);
}

ec_status ec_batch_reserve(ec_batch *b, int n_stripes, size_t n_items) {
  if (!b || n_stripes < 0) return EC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return EC_ERR_DEVICE;
  return grow(b, (size_t)n_stripes, 2 * n_items);
}

ec_status ec_batch_build(const ec_stripe *stripes, int n_stripes, size_t tile_bytes, ec_stream stream,
                         ec_batch **out) {
  if (!out) return EC_ERR_ARG;
  *out = nullptr;
  ec_batch *raw = nullptr;
  ec_status st = ec_batch_create(&raw);
  if (st != EC_OK) return st;
  std::unique_ptr<ec_batch> b(raw);
  st = ec_batch_set(b.get(), stripes, n_stripes, tile_bytes, stream);
  if (st != EC_OK) return st;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return EC_ERR_DEVICE;
  // Capture the persistent kernel into a graph on a private stream.
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return EC_ERR_DEVICE;
  bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
  ok = ok && batch_launch(b->slots, b->args, b->grid, cap) == 0;
  ok = (hipStreamEndCapture(cap, &b->graph) == hipSuccess) && ok;
  ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  (void)hipStreamDestroy(cap);
  if (!ok) return EC_ERR_DEVICE;
  *out = b.release();
  return EC_OK;
}

ec_status ec_batch_launch(ec_batch *batch, ec_stream stream) {
  if (!batch || !batch->exec) return EC_ERR_ARG;
  return hipGraphLaunch(batch->exec, (hipStream_t)stream) == hipSuccess ? EC_OK : EC_ERR_DEVICE;
}

ec_status ec_batch_enqueue(ec_batch *batch, ec_stream stream) {
  if (!batch || batch->n_items == 0) return EC_ERR_ARG;
  return batch_launch(batch->slots, batch->args, batch->grid, (hipStream_t)stream) == 0 ? EC_OK : EC_ERR_DEVICE;
}

ec_status ec_batch_query(const ec_batch *batch, size_t *n_items, size_t *in_bytes, size_t *out_bytes) {
  if (!batch) return EC_ERR_ARG;
  if (n_items) *n_items = batch->n_items;
  if (in_bytes) *in_bytes = batch->in_bytes;
  if (out_bytes) *out_bytes = batch->out_bytes;
  return EC_OK;
}

void ec_batch_free(ec_batch *batch) { delete batch; }

}  // extern "C"
