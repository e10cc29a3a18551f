// program_pool.cpp -- the per-device pool of program images.
#include "program_pool.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "arena.hpp"

namespace ec {

namespace {

constexpr size_t kChunkBytes = 4u << 20;  // smallest chunk allocated
constexpr size_t kAlign = 256;            // image placement granule

struct Chunk {
  uint8_t *base = nullptr;
  size_t bytes = 0;
  FirstFit heap;
  size_t used = 0;
  Chunk(uint8_t *b, size_t n) : base(b), bytes(n), heap(n, kAlign) {}
};

struct Image {
  std::vector<uint32_t> words;  // host copy, to tell images with equal hashes apart
  uint32_t *dev = nullptr;
  size_t chunk = 0, off = 0, got = 0;
  int refs = 0;
};

struct DevicePool {
  std::mutex mu;
  std::vector<std::unique_ptr<Chunk>> chunks;
  std::unordered_multimap<uint64_t, std::unique_ptr<Image>> by_hash;
  std::map<const uint32_t *, Image *> by_ptr;
};

// Never destroyed: programs may be freed while the process exits.
std::mutex *const g_mu = new std::mutex;
std::map<int, std::unique_ptr<DevicePool>> *const g_pools = new std::map<int, std::unique_ptr<DevicePool>>;

DevicePool &pool_of(int dev) {
  std::lock_guard<std::mutex> g(*g_mu);
  auto &p = (*g_pools)[dev];
  if (!p) p.reset(new DevicePool);
  return *p;
}

// FNV-1a over the words
uint64_t hash_words(const std::vector<uint32_t> &w) {
  uint64_t h = 1469598103934665603ull;
  for (uint32_t x : w) {
    for (int k = 0; k < 4; ++k) {
      h ^= (x >> (8 * k)) & 0xFFu;
      h *= 1099511628211ull;
    }
  }
  return h ^ w.size();
}

// A piece of `bytes` in some chunk (a new chunk of at least kChunkBytes if
// none has room); false if the device allocation fails.
bool place(DevicePool &p, size_t bytes, size_t *chunk, size_t *off, size_t *got) {
  for (size_t c = 0; c < p.chunks.size(); ++c) {
    const size_t o = p.chunks[c]->heap.alloc(bytes, got);
    if (o != SIZE_MAX) {
      *chunk = c;
      *off = o;
      p.chunks[c]->used += *got;
      return true;
    }
  }
  const size_t n = std::max(kChunkBytes, (bytes + kAlign - 1) / kAlign * kAlign);
  uint8_t *d = nullptr;
  if (hipMalloc((void **)&d, n) != hipSuccess) return false;
  p.chunks.emplace_back(new Chunk(d, n));
  *chunk = p.chunks.size() - 1;
  *off = p.chunks.back()->heap.alloc(bytes, got);
  p.chunks.back()->used += *got;
  return *off != SIZE_MAX;
}

}  // namespace

const uint32_t *pool_acquire(int dev, const std::vector<uint32_t> &image, ec_status *st) {
  DevicePool &p = pool_of(dev);
  std::lock_guard<std::mutex> g(p.mu);
  const uint64_t h = hash_words(image);
  auto range = p.by_hash.equal_range(h);
  for (auto it = range.first; it != range.second; ++it)
    if (it->second->words == image) {
      ++it->second->refs;
      return it->second->dev;
    }
  const size_t bytes = image.size() * sizeof(uint32_t);
  std::unique_ptr<Image> im(new Image);
  if (!place(p, bytes, &im->chunk, &im->off, &im->got)) {
    *st = EC_ERR_NOMEM;
    return nullptr;
  }
  im->dev = (uint32_t *)(p.chunks[im->chunk]->base + im->off);
  if (hipMemcpy(im->dev, image.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    p.chunks[im->chunk]->heap.release(im->off, im->got);
    p.chunks[im->chunk]->used -= im->got;
    *st = EC_ERR_DEVICE;
    return nullptr;
  }
  im->words = image;
  im->refs = 1;
  Image *raw = im.get();
  p.by_ptr[raw->dev] = raw;
  p.by_hash.emplace(h, std::move(im));
  return raw->dev;
}

void pool_release(int dev, const uint32_t *words) {
  DevicePool &p = pool_of(dev);
  std::lock_guard<std::mutex> g(p.mu);
  auto it = p.by_ptr.find(words);
  if (it == p.by_ptr.end()) return;
  Image *im = it->second;
  if (--im->refs > 0) return;
  p.chunks[im->chunk]->heap.release(im->off, im->got);
  p.chunks[im->chunk]->used -= im->got;
  p.by_ptr.erase(it);
  const uint64_t h = hash_words(im->words);
  auto range = p.by_hash.equal_range(h);
  for (auto jt = range.first; jt != range.second; ++jt)
    if (jt->second.get() == im) {
      p.by_hash.erase(jt);
      break;
    }
}

size_t pool_missing_bytes(int dev, const std::vector<const std::vector<uint32_t> *> &images) {
  DevicePool &p = pool_of(dev);
  std::lock_guard<std::mutex> g(p.mu);
  std::unordered_multimap<uint64_t, const std::vector<uint32_t> *> seen;
  size_t bytes = 0;
  for (const std::vector<uint32_t> *w : images) {
    const uint64_t h = hash_words(*w);
    bool have = false;
    auto range = p.by_hash.equal_range(h);
    for (auto it = range.first; it != range.second && !have; ++it) have = it->second->words == *w;
    auto mine = seen.equal_range(h);
    for (auto it = mine.first; it != mine.second && !have; ++it) have = *it->second == *w;
    if (have) continue;
    seen.emplace(h, w);
    bytes += (w->size() * sizeof(uint32_t) + kAlign - 1) / kAlign * kAlign;
  }
  return bytes;
}

ec_status pool_reserve(int dev, size_t bytes) {
  DevicePool &p = pool_of(dev);
  std::lock_guard<std::mutex> g(p.mu);
  for (auto &c : p.chunks)
    for (const auto &r : c->heap.free_ranges())
      if (r.second >= bytes) return EC_OK;
  const size_t n = std::max(kChunkBytes, (bytes + kAlign - 1) / kAlign * kAlign);
  uint8_t *d = nullptr;
  if (hipMalloc((void **)&d, n) != hipSuccess) return EC_ERR_NOMEM;
  p.chunks.emplace_back(new Chunk(d, n));
  return EC_OK;
}

void pool_stats(int dev, int *chunks, int *images, size_t *bytes_used) {
  DevicePool &p = pool_of(dev);
  std::lock_guard<std::mutex> g(p.mu);
  size_t used = 0;
  for (auto &c : p.chunks) used += c->used;
  if (chunks) *chunks = (int)p.chunks.size();
  if (images) *images = (int)p.by_ptr.size();
  if (bytes_used) *bytes_used = used;
}

}  // namespace ec
