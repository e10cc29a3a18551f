// serve.cpp -- the serving loop: continuous batching of encode and decode
// requests under an HBM budget, run on the caller's thread.
//
// Requests arrive on the caller's clock (arrival times relative to the start
// of a run).  The loop admits arrived requests while their inputs and
// outputs fit the budget and their outputs fit a first-fit arena, spreads
// them over the free slots and packs each slot's share into one launch on
// that slot's stream (a plain launch for a single request, a reusable batch
// otherwise), and keeps admitting while earlier launches run, so work
// admitted meanwhile overlaps on the device.  It polls each busy slot's
// event and records completion times on the same clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <map>
#include <memory>
#include <new>
#include <set>
#include <vector>

#include "../../include/ec.h"
#include "arena.hpp"
#include "batch.hpp"
#include "exec.hpp"
#include "program.hpp"

using namespace ec;

namespace {

constexpr size_t kArenaAlign = 4096;  // output placement granule
constexpr int kMaxSlots = 16;
constexpr size_t kWarmBlock = 128;    // block bytes of the warm-up launches

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct ec_server {
  int device = 0;
  uint8_t *arena = nullptr;
  size_t arena_bytes = 0;
  size_t budget = 0;
  int max_batch = 1;
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ec_batch *batch = nullptr;
    std::vector<int> reqs;  // requests in flight on this slot (empty: free)
  };
  std::vector<Slot> slots;
  std::set<int> warmed;  // slot budgets whose kernels have run on every stream

  ~ec_server() {
    int cur = 0;
    const bool swap = hipGetDevice(&cur) == hipSuccess && cur != device && hipSetDevice(device) == hipSuccess;
    for (Slot &s : slots) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.batch) ec_batch_free(s.batch);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    if (swap) (void)hipSetDevice(cur);
  }
};

namespace {

size_t n_out_of(const ec_program *p) { return p->out_blocks.size(); }
size_t n_in_of(const ec_program *p) { return p->in_blocks.size(); }

ec_status launch_one(const ec_program *prog, const uint8_t *const *in, uint8_t *const *out, size_t bb,
                     hipStream_t s) {
  return prog->decode ? ec_decode(prog, in, out, bb, (ec_stream)s) : ec_encode(prog, in, out, bb, (ec_stream)s);
}

// One tiny direct launch and one tiny batch of `prog` on every slot's
// stream: the first launches on a new stream, and of each kernel, take
// milliseconds, which the first requests would otherwise wait for.  Blocks
// of kWarmBlock bytes at the start of the arena serve as inputs and outputs
// (nothing is placed there yet).
ec_status warm(ec_server *sv, const ec_program *prog) {
  const size_t ni = n_in_of(prog), no = n_out_of(prog);
  std::vector<const uint8_t *> in(ni);
  std::vector<uint8_t *> out(no);
  for (size_t i = 0; i < ni; ++i) in[i] = sv->arena + i * kWarmBlock;
  for (size_t j = 0; j < no; ++j) out[j] = sv->arena + (ni + j) * kWarmBlock;
  for (auto &s : sv->slots) {
    ec_status st = launch_one(prog, in.data(), out.data(), kWarmBlock, s.stream);
    if (st != EC_OK) return st;
    const ec_stripe one{prog, in.data(), out.data(), kWarmBlock};
    st = ec_batch_set(s.batch, &one, 1, 0, (ec_stream)s.stream);
    if (st == EC_OK) st = ec_batch_enqueue(s.batch, (ec_stream)s.stream);
    if (st != EC_OK) return st;
  }
  for (auto &s : sv->slots)
    if (hipStreamSynchronize(s.stream) != hipSuccess) return EC_ERR_DEVICE;
  return EC_OK;
}

}  // namespace

extern "C" {

ec_status ec_server_create(uint8_t *arena, size_t arena_bytes, const ec_serve_opts *opts, ec_server **out) {
  if (!out) return EC_ERR_ARG;
  *out = nullptr;
  if (!arena || !opts || opts->budget_bytes == 0 || opts->n_slots < 1 || opts->n_slots > kMaxSlots ||
      opts->max_batch < 1)
    return EC_ERR_ARG;
  if (((uintptr_t)arena & 15u) != 0) return EC_ERR_ALIGN;
  if (arena_bytes < (size_t)kMaxBlocks * kWarmBlock) return EC_ERR_ARG;
  std::unique_ptr<ec_server> sv(new (std::nothrow) ec_server);
  if (!sv) return EC_ERR_NOMEM;
  if (hipGetDevice(&sv->device) != hipSuccess) return EC_ERR_DEVICE;
  sv->arena = arena;
  sv->arena_bytes = arena_bytes;
  sv->budget = opts->budget_bytes;
  sv->max_batch = opts->max_batch;
  sv->slots.resize((size_t)opts->n_slots);
  for (auto &s : sv->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return EC_ERR_DEVICE;
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return EC_ERR_DEVICE;
    const ec_status st = ec_batch_create(&s.batch);
    if (st != EC_OK) return st;
  }
  *out = sv.release();
  return EC_OK;
}

ec_status ec_server_run(ec_server *sv, const ec_request *reqs, int n_reqs, int realtime, ec_serve_done_fn on_done,
                        void *user, double *done_s, size_t *out_offsets, double *wall_s, int *n_batches) {
  if (!sv || n_reqs < 0 || (n_reqs > 0 && (!reqs || !done_s))) return EC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != sv->device) return EC_ERR_DEVICE;
  const size_t n = (size_t)n_reqs;
  // Check every request up front: a request that could never be admitted
  // would otherwise stall the loop.  Outputs are placed in the arena, disjoint
  // from each other by construction, so an input outside the arena is all
  // that keeps every launch free of overlaps (the launches then skip that
  // check).
  size_t max_tiles = 1;
  std::vector<const ec_program *> progs;
  const uintptr_t arena_lo = (uintptr_t)sv->arena, arena_hi = arena_lo + sv->arena_bytes;
  for (size_t i = 0; i < n; ++i) {
    const ec_request &r = reqs[i];
    if (!r.prog || !r.in || !std::isfinite(r.arrival_s) || r.arrival_s < 0) return EC_ERR_ARG;
    if (i > 0 && r.arrival_s < reqs[i - 1].arrival_s) return EC_ERR_ARG;
    if (r.block_bytes == 0 || r.block_bytes % 128 != 0) return EC_ERR_ALIGN;
    if (r.block_bytes / 8 > 0x1FFFFFFFull) return EC_ERR_UNSUPPORTED;
    for (size_t k = 0; k < n_in_of(r.prog); ++k) {
      const uintptr_t a = (uintptr_t)r.in[k];
      if (!a) return EC_ERR_ARG;
      if (a & 15u) return EC_ERR_ALIGN;
      if (a < arena_hi && arena_lo < a + r.block_bytes) return EC_ERR_ARG;
    }
    const size_t out_bytes = n_out_of(r.prog) * r.block_bytes;
    if (out_bytes == 0) return EC_ERR_ARG;
    if ((n_in_of(r.prog) + n_out_of(r.prog)) * r.block_bytes > sv->budget) return EC_ERR_CAPACITY;
    if ((out_bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign > sv->arena_bytes) return EC_ERR_CAPACITY;
    max_tiles = std::max(max_tiles, (r.block_bytes / 8 + kTileBytes - 1) / kTileBytes);
    progs.push_back(r.prog);
  }
  // Programs on the device, tables sized and kernels warmed before the clock
  // starts: nothing below allocates.
  std::sort(progs.begin(), progs.end());
  progs.erase(std::unique(progs.begin(), progs.end()), progs.end());
  {
    // one device allocation at most for all of them
    std::vector<ec_program *> mut;
    for (const ec_program *p : progs) mut.push_back(const_cast<ec_program *>(p));
    const ec_status st = ec_program_upload_many(mut.data(), (int)mut.size());
    if (st != EC_OK) return st;
  }
  // Work items of one batch: at most one per tile of each request's strips,
  // or, with a row split, one per resident wave (fewer than 8192).
  const size_t max_items = std::max<size_t>(8192, (size_t)sv->max_batch * (max_tiles + 1));
  for (auto &s : sv->slots) {
    const ec_status st = ec_batch_reserve(s.batch, sv->max_batch, max_items);
    if (st != EC_OK) return st;
  }
  for (const ec_program *p : progs)
    if (!sv->warmed.count(p->slots)) {
      const ec_status st = warm(sv, p);
      if (st != EC_OK) return st;
      sv->warmed.insert(p->slots);
    }

  FirstFit heap(sv->arena_bytes, kArenaAlign);
  std::vector<size_t> out_off(n, 0), out_len(n, 0);
  std::vector<uint8_t *> outs;  // output pointers of the batch being launched
  std::vector<ec_stripe> stripes;
  std::vector<int> ids;
  std::vector<size_t> offs;
  outs.reserve((size_t)sv->max_batch * kMaxBlocks);
  stripes.reserve((size_t)sv->max_batch);
  size_t used = 0, next = 0, finished = 0;
  int batches = 0;
  ec_status err = EC_OK;
  const double t0 = now_s();

  auto bytes_of = [&](size_t i) { return (n_in_of(reqs[i].prog) + n_out_of(reqs[i].prog)) * reqs[i].block_bytes; };
  auto retire = [&]() -> ec_status {
    for (auto &s : sv->slots) {
      if (s.reqs.empty()) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return EC_ERR_DEVICE;
      const double t = now_s() - t0;
      for (int r : s.reqs) done_s[r] = t;
      if (on_done) {
        ids.assign(s.reqs.begin(), s.reqs.end());
        offs.clear();
        for (int r : s.reqs) offs.push_back(out_off[(size_t)r]);
        on_done(user, ids.data(), (int)ids.size(), offs.data());
      }
      for (int r : s.reqs) {
        heap.release(out_off[(size_t)r], out_len[(size_t)r]);
        used -= bytes_of((size_t)r);
      }
      finished += s.reqs.size();
      s.reqs.clear();
    }
    return EC_OK;
  };
  auto launch = [&](ec_server::Slot &s) -> ec_status {
    // every output pointer first (outs never grows past its reserved size,
    // so the stripes' pointers into it stay valid), then the stripes
    outs.clear();
    stripes.clear();
    for (int r : s.reqs) {
      const ec_request &q = reqs[(size_t)r];
      for (size_t j = 0; j < n_out_of(q.prog); ++j) outs.push_back(sv->arena + out_off[(size_t)r] + j * q.block_bytes);
    }
    size_t k = 0;
    for (int r : s.reqs) {
      const ec_request &q = reqs[(size_t)r];
      stripes.push_back(ec_stripe{q.prog, q.in, outs.data() + k, q.block_bytes});
      k += n_out_of(q.prog);
    }
    ec_status st;
    if (stripes.size() == 1) {
      // one request: a plain launch, without the batch's tables and work counter
      st = launch_one(stripes[0].prog, stripes[0].in, stripes[0].out, stripes[0].block_bytes, s.stream);
    } else {
      st = batch_set(s.batch, stripes.data(), (int)stripes.size(), 0, (ec_stream)s.stream, false);
      if (st == EC_OK) st = ec_batch_enqueue(s.batch, (ec_stream)s.stream);
    }
    if (st != EC_OK) return st;
    if (hipEventRecord(s.done, s.stream) != hipSuccess) return EC_ERR_DEVICE;
    ++batches;
    return EC_OK;
  };

  while (finished < n) {
    if ((err = retire()) != EC_OK) break;
    ec_server::Slot *slot = nullptr;
    size_t n_free = 0;
    for (auto &s : sv->slots)
      if (s.reqs.empty()) {
        if (!slot) slot = &s;
        ++n_free;
      }
    if (!slot || next >= n) continue;
    const double now = realtime ? now_s() - t0 : INFINITY;
    // The arrived requests' work (bytes read and written; looking at most
    // max_batch requests per free slot ahead) is spread evenly over the free
    // slots: a request launched alone on its own stream finishes sooner than
    // in a batch with others, while a backlog is cut into launches of equal
    // work, each of up to max_batch requests.
    size_t arrived = 0, arrived_bytes = 0;
    const size_t cap = n_free * (size_t)sv->max_batch;
    while (next + arrived < n && reqs[next + arrived].arrival_s <= now && arrived < cap) {
      arrived_bytes += bytes_of(next + arrived);
      ++arrived;
    }
    const size_t share = (arrived_bytes + n_free - 1) / n_free;
    // Arrived requests that fit, in arrival order, until this launch holds
    // its share of the work or max_batch requests, all of one slot budget
    // (one kernel instance per batch).
    int kslots = -1;
    size_t launch_bytes = 0;
    while (next < n && reqs[next].arrival_s <= now && slot->reqs.size() < (size_t)sv->max_batch &&
           (slot->reqs.empty() || launch_bytes < share)) {
      const ec_request &q = reqs[next];
      if (kslots >= 0 && q.prog->slots != kslots) break;
      if (used + bytes_of(next) > sv->budget) break;
      size_t got = 0;
      const size_t off = heap.alloc(n_out_of(q.prog) * q.block_bytes, &got);
      if (off == SIZE_MAX) break;
      out_off[next] = off;
      out_len[next] = got;
      used += bytes_of(next);
      kslots = q.prog->slots;
      launch_bytes += bytes_of(next);
      slot->reqs.push_back((int)next);
      ++next;
    }
    if (!slot->reqs.empty() && (err = launch(*slot)) != EC_OK) break;
  }
  if (err != EC_OK) {
    // leave nothing running on the caller's buffers
    for (auto &s : sv->slots) {
      (void)hipStreamSynchronize(s.stream);
      s.reqs.clear();
    }
    return err;
  }
  if (wall_s) *wall_s = now_s() - t0;
  if (out_offsets) std::copy(out_off.begin(), out_off.end(), out_offsets);
  if (n_batches) *n_batches = batches;
  return EC_OK;
}

void ec_server_free(ec_server *sv) { delete sv; }

}  // extern "C"
