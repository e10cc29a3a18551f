// noalloc.hip -- the batched launch for callers that cannot allocate.
//
// ec_batch_run_noalloc is ec_batch_set + ec_batch_enqueue in one call, with
// the batch's device tables (work counter, stripe descriptors, work items)
// in `scratch`, a fixed array of EC_NOALLOC_SCRATCH_BYTES per device, instead
// of memory the library allocates.  The host side stages the tables in a
// static host array of the same layout and copies them with hipMemcpyAsync;
// nothing is allocated on the host or the device.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is taken once per device with hipGetSymbolAddress, and
// only that address is used (copy destination, kernel arguments).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ec.h"
#include "batch.hpp"
#include "exec.hpp"

using namespace ec;

namespace {

static __device__ __align__(256) uint8_t scratch[EC_NOALLOC_SCRATCH_BYTES];

// Layout of the scratch array (and of the host staging array):
//   [0, 256)                   the work counter;
//   [kDescOff, kItemsOff)      EC_NOALLOC_MAX_STRIPES stripe descriptors;
//   [kItemsOff, end)           work items, two 32-bit words each.
constexpr size_t kDescOff = 256;
constexpr size_t kItemsOff = (kDescOff + EC_NOALLOC_MAX_STRIPES * sizeof(StripeDesc) + 255) / 256 * 256;
static_assert(kItemsOff < EC_NOALLOC_SCRATCH_BYTES, "scratch too small for the descriptors");
constexpr uint64_t kMaxItems = (EC_NOALLOC_SCRATCH_BYTES - kItemsOff) / (2 * sizeof(uint32_t));
// Block ranges of a launch: at most kMaxBlocks per stripe.
constexpr size_t kMaxRanges = (size_t)EC_NOALLOC_MAX_STRIPES * kMaxBlocks;

constexpr int kMaxDevices = 64;

// Everything below is guarded by g_mu: the host staging and the range
// workspaces are shared by every call, and a call holds the lock until its
// copy has consumed the staging (a copy from pageable host memory returns
// once its source has been read).
std::mutex g_mu;
uint8_t *g_scratch[kMaxDevices];  // device address of `scratch` on each device (null: not taken yet)
int g_cus[kMaxDevices];
alignas(256) uint8_t g_stage[EC_NOALLOC_SCRATCH_BYTES];
ByteRange g_reads[kMaxRanges], g_writes[kMaxRanges];

// The current device's scratch address and compute units, looked up on the
// first call on that device (with it current).
ec_status device_scratch(int *device, uint8_t **ptr, int *n_cus) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EC_ERR_DEVICE;
  *device = dev;
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EC_ERR_DEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      return EC_ERR_DEVICE;
    g_cus[dev] = cus;
    g_scratch[dev] = (uint8_t *)p;
  }
  *ptr = g_scratch[dev];
  *n_cus = g_cus[dev];
  return EC_OK;
}

}  // namespace

extern "C" ec_status ec_batch_run_noalloc(const ec_stripe *stripes, int n_stripes, size_t tile_bytes,
                                          ec_stream stream) {
  if (!stripes || n_stripes <= 0) return EC_ERR_ARG;
  if (n_stripes > EC_NOALLOC_MAX_STRIPES) return EC_ERR_CAPACITY;
  std::lock_guard<std::mutex> g(g_mu);
  uint8_t *dev = nullptr;
  int device = 0, n_cus = 0;
  ec_status st = device_scratch(&device, &dev, &n_cus);
  if (st != EC_OK) return st;
  BatchPlan plan;
  st = batch_plan(stripes, n_stripes, tile_bytes, n_cus, &plan);
  if (st != EC_OK) return st;
  if (plan.n_items > kMaxItems) return EC_ERR_CAPACITY;
  StripeDesc *desc = (StripeDesc *)(g_stage + kDescOff);
  uint32_t *items = (uint32_t *)(g_stage + kItemsOff);
  st = batch_fill(stripes, n_stripes, plan, device, false, desc, items, g_reads, g_writes);
  if (st != EC_OK) return st;
  // The descriptors and the items (the counter is reset by the launch's own
  // first kernel, not by a copy or a memset).
  const hipStream_t hs = (hipStream_t)stream;
  if (hipMemcpyAsync(dev + kDescOff, desc, (size_t)n_stripes * sizeof(StripeDesc), hipMemcpyHostToDevice, hs) !=
          hipSuccess ||
      hipMemcpyAsync(dev + kItemsOff, items, plan.n_items * 2 * sizeof(uint32_t), hipMemcpyHostToDevice, hs) !=
          hipSuccess)
    return EC_ERR_DEVICE;
  BatchArgs a{};
  a.stripes = (const StripeDesc *)(dev + kDescOff);
  a.items = (const uint32_t *)(dev + kItemsOff);
  a.n_items = (uint32_t)plan.n_items;
  a.tiles_per_item = plan.tiles_per_item;
  a.chunk = 1;
  a.counter = (uint32_t *)dev;
  return batch_launch(plan.slots, a, batch_grid(plan, n_cus), hs) == 0 ? EC_OK : EC_ERR_DEVICE;
}
