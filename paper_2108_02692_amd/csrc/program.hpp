// program.hpp -- the library-internal layout of a compiled program.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/ec.h"
#include "native.hpp"
#include "program_pool.hpp"
#include "push.hpp"
#include "slp.hpp"

struct ec_program {
  // one compiled program: host IR of every stage, the bytecode, and its
  // per-device copies
  int n = 0, p = 0;
  bool decode = false;
  int level = EC_LEVEL_CO_FU_SCHED;
  int slots = 32;
  std::vector<int> in_blocks, out_blocks;
  ec::Slp plain, co, fu, sched;  // the paper's whole-matrix stages (co/fu/sched per level)
  std::vector<ec::Bits> brows;   // the bitmatrix rows (input of the stages)
  bool rebuild = true;           // XorRePair (else RePair)
  bool stages_built = false;
  ec::Slp exec;                  // the push-form program the executor runs, as an SLP
  ec::PushCode code;
  std::vector<ec::PushCode> parts;      // row-split parts of whole output blocks (empty: none)
  std::vector<ec::PushCode> row_parts;   // row-split parts of single rows or small row groups
  std::vector<ec::PushCode> pair_parts;  // row-split parts of row pairs (or small groups of pairs)
  std::vector<ec::PushCode> pass_parts;  // one pass each, when the program needs several (empty: none)
  std::vector<ec::PushCode> stage_parts; // runs of rows for the staged launch (EC_SPLIT_STAGED only)
  std::vector<uint32_t> image;           // device image: code.words, then parts, row_parts, pair_parts, pass_parts, stage_parts
  std::vector<uint32_t> part_off;        // word offset of each part in the image
  std::vector<uint32_t> row_part_off;    // word offset of each row part in the image
  std::vector<uint32_t> pair_part_off;   // word offset of each pair part in the image
  std::vector<uint32_t> pass_part_off;   // word offset of each pass part in the image
  std::vector<uint32_t> stage_part_off;  // word offset of each stage part in the image
  // native kernels (empty: none): [0] the whole program, [1] its pair
  // parts, [2] its block parts; kernel k is compiled for EC_NATIVE_* bit 1 << k
  std::string native_src[ec::kNativeKernels];
  std::vector<char> native_code[ec::kNativeKernels];
  std::map<std::pair<int, int>, std::pair<hipFunction_t, int>> native_fn;  // (device, kernel) -> kernel, workgroups per CU
  int split = EC_SPLIT_AUTO;
  ec_program_info info{};
  std::mutex mu;
  std::map<int, const uint32_t *> dev_words;  // device -> bytecode copy (in the device's program pool)
  // the same pointers for the first kDevCache device ids, read without the
  // lock (a batch looks up every stripe's program on every launch)
  static constexpr int kDevCache = 16;
  std::atomic<const uint32_t *> dev_cache[kDevCache] = {};

  ~ec_program() {
    for (auto &kv : dev_words) ec::pool_release(kv.first, kv.second);
  }

  // Native kernel `which` (0 whole program, 1 pair parts, 2 block parts) on device `dev`
  // (the current device), loaded on first use; null and *st set if it
  // cannot be loaded.
  hipFunction_t native_function(int dev, int which, int *per_cu, ec_status *st) {
    std::lock_guard<std::mutex> g(mu);
    auto it = native_fn.find({dev, which});
    if (it == native_fn.end()) {
      hipFunction_t fn = nullptr;
      int n = 0;
      *st = ec::native_function(dev, native_code[which], &fn, &n);
      if (*st != EC_OK) return nullptr;
      it = native_fn.emplace(std::make_pair(dev, which), std::make_pair(fn, n)).first;
    }
    *per_cu = it->second.second;
    return it->second.first;
  }

  // Builds the whole-matrix CO/FU/SCHED stages of the program's level once.
  void paper_stages() {
    std::lock_guard<std::mutex> g(mu);
    if (stages_built) return;
    const int n_const = plain.n_const;
    if (level >= EC_LEVEL_CO) co = ec::xor_repair(brows, n_const, rebuild);
    if (level >= EC_LEVEL_CO_FU) fu = ec::fuse(co);
    if (level >= EC_LEVEL_CO_FU_SCHED) sched = ec::dfs_schedule(fu);
    stages_built = true;
  }

  // The device copy of the bytecode on device `dev`, or null if it has not
  // been uploaded there (allocates nothing).
  const uint32_t *device_words_present(int dev) {
    if (dev >= 0 && dev < kDevCache) {
      const uint32_t *p = dev_cache[dev].load(std::memory_order_acquire);
      if (p) return p;
    }
    std::lock_guard<std::mutex> g(mu);
    auto it = dev_words.find(dev);
    return it == dev_words.end() ? nullptr : it->second;
  }

  // Device copy of the bytecode for the current device (uploaded once).
  const uint32_t *device_words(ec_status *st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { *st = EC_ERR_DEVICE; return nullptr; }
    return device_words(dev, st);
  }

  // Device copy of the bytecode for device `dev`, the current device
  // (placed in the device's program pool once, shared with identical
  // images).
  const uint32_t *device_words(int dev, ec_status *st) {
    if (const uint32_t *p = device_words_present(dev)) return p;
    std::lock_guard<std::mutex> g(mu);
    auto it = dev_words.find(dev);
    if (it != dev_words.end()) return it->second;
    const uint32_t *d = ec::pool_acquire(dev, image, st);
    if (!d) return nullptr;
    dev_words[dev] = d;
    if (dev >= 0 && dev < kDevCache) dev_cache[dev].store(d, std::memory_order_release);
    return d;
  }
};

