// The library's host side (matrices, the compile pipeline, inspection and
// argument checking) run under AddressSanitizer and UndefinedBehaviorSanitizer.
// Built with g++ from the library's C++ sources; the device launchers are
// replaced by stubs below, and no call here reaches the HIP runtime.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/ec.h"
#include "../../paper_2108_02692_amd/csrc/arena.hpp"
#include "../../paper_2108_02692_amd/csrc/exec.hpp"

namespace ec {
int exec_launch(int, const ExecArgs &, int, hipStream_t) { return -1; }
int batch_launch(int, const BatchArgs &, int, hipStream_t) { return -1; }
int copy_launch(const void *, void *, uint64_t, int, hipStream_t) { return -1; }
int stream_launch(const ExecArgs &, uint32_t, int, hipStream_t) { return -1; }
int staged_launch(int, const ExecArgs &, int, uint32_t, hipStream_t) { return -1; }
}  // namespace ec

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

// paper_stages: also export the whole-matrix stages of Secs. 4-6 and the
// greedy schedule (slow under the sanitizers, so only for some programs).
static void exercise(const ec_program *prog, int level, bool paper_stages) {
  ec_program_info info;
  CHECK(ec_program_query(prog, &info) == EC_OK);
  const uint32_t *words = nullptr;
  size_t n_words = 0;
  CHECK(ec_program_bytecode(prog, &words, &n_words) == EC_OK && n_words == info.n_words);
  for (int stage = EC_STAGE_PLAIN; stage <= EC_STAGE_EXEC; ++stage) {
    if (!paper_stages && stage >= EC_STAGE_CO && stage <= EC_STAGE_SCHED) continue;
    const bool have = stage == EC_STAGE_PLAIN || stage == EC_STAGE_EXEC || level >= stage;
    size_t len = 0;
    const ec_status st = ec_program_export(prog, stage, nullptr, 0, &len);
    CHECK((st == EC_OK) == have);
    if (st != EC_OK) continue;
    std::vector<int32_t> buf(len);
    CHECK(ec_program_export(prog, stage, buf.data(), len, &len) == EC_OK && len == buf.size());
    if (len > 4) {  // a short buffer is filled only up to its capacity
      std::vector<int32_t> part(4, 7);
      CHECK(ec_program_export(prog, stage, part.data(), 3, &len) == EC_OK && part[3] == 7);
    }
  }
  for (int cap : {1, 8, 64}) {
    if (!paper_stages) break;
    size_t len = 0;
    const ec_status st = ec_program_export_greedy(prog, cap, nullptr, 0, &len);
    CHECK((st == EC_OK) == (level >= EC_LEVEL_CO_FU));
    if (st == EC_OK) {
      std::vector<int32_t> buf(len);
      CHECK(ec_program_export_greedy(prog, cap, buf.data(), len, &len) == EC_OK);
    }
  }
  // launch argument checks that fail before any device call
  std::vector<const uint8_t *> in(info.n_in, nullptr);
  std::vector<uint8_t *> out(info.n_out, nullptr);
  CHECK(ec_encode(prog, in.data(), out.data(), 4096, nullptr) != EC_OK);
  CHECK(ec_decode(prog, nullptr, out.data(), 4096, nullptr) == EC_ERR_ARG);
}

int main() {
  struct Codec { int n, p; } codecs[] = {{6, 3}, {10, 4}, {12, 4}, {14, 4}, {1, 0}, {1, 1}, {2, 1}, {28, 4}, {8, 2}};
  unsigned seed = 12345;
  int compiled = 0;
  for (const Codec &c : codecs) {
    std::vector<uint8_t> gen((size_t)(c.n + c.p) * c.n);
    CHECK(ec_matrix_cauchy(c.n, c.p, gen.data()) == EC_OK);
    for (int level = EC_LEVEL_PLAIN; level <= EC_LEVEL_CO_FU_SCHED; ++level) {
      for (int budget : {0, 24, 48}) {
        if (budget && c.n != 10) continue;  // other budgets on RS(10,4) only
        // the encode, then a few random erasure sets of 1..p blocks
        for (int t = 0; t < 1 + 2 * (c.p > 0); ++t) {
          std::vector<int> er;
          if (t > 0) {
            const int k = 1 + (int)(seed = seed * 1103515245u + 12345u) % c.p;
            while ((int)er.size() < k) {
              const int e = (int)((seed = seed * 1103515245u + 12345u) >> 8) % (c.n + c.p);
              bool dup = false;
              for (int x : er) dup |= x == e;
              if (!dup) er.push_back(e);
            }
          }
          ec_compile_opts o{};
          o.level = (uint32_t)level;
          o.slot_budget = (uint32_t)budget;
          // now and then one block over the whole matrix (not for the widest
          // codec, whose whole-matrix compression is slow under the sanitizers)
          o.block_strips = (uint32_t)((seed >> 4) % 3 == 0 && c.n <= 14 ? 8 * c.n : 0);
          ec_program *prog = nullptr;
          const ec_status st = ec_compile_slp(c.n, c.p, gen.data(), er.data(), (int)er.size(), &o, &prog);
          CHECK(st == EC_OK || st == EC_ERR_CAPACITY);
          if (st != EC_OK) continue;
          exercise(prog, level, budget == 0 && t <= 1 && c.n <= 14);
          ec_program_free(prog);
          ++compiled;
        }
      }
    }
  }
  // the paper-reading generator and the RePair variant
  {
    std::vector<uint8_t> gen(14 * 10);
    CHECK(ec_matrix_vandermonde(10, 4, gen.data()) == EC_OK);
    ec_compile_opts o{};
    o.level = EC_LEVEL_CO_FU_SCHED;
    o.compress = EC_COMPRESS_REPAIR;
    const int er[] = {2, 4, 5, 6};
    ec_program *prog = nullptr;
    CHECK(ec_compile_slp(10, 4, gen.data(), er, 4, &o, &prog) == EC_OK);
    if (prog) exercise(prog, EC_LEVEL_CO_FU_SCHED, true), ec_program_free(prog);
  }
  // argument errors
  {
    std::vector<uint8_t> gen(14 * 10);
    ec_matrix_cauchy(10, 4, gen.data());
    ec_program *prog = nullptr;
    const int five[] = {0, 1, 2, 3, 4}, dup[] = {1, 1}, bad[] = {14};
    CHECK(ec_compile_slp(10, 4, gen.data(), five, 5, nullptr, &prog) == EC_ERR_TOO_MANY_ERASURES);
    CHECK(ec_compile_slp(10, 4, gen.data(), dup, 2, nullptr, &prog) == EC_ERR_ARG);
    CHECK(ec_compile_slp(10, 4, gen.data(), bad, 1, nullptr, &prog) == EC_ERR_ARG);
    CHECK(ec_compile_slp(10, 4, nullptr, nullptr, 0, nullptr, &prog) == EC_ERR_ARG);
    CHECK(ec_compile_slp(10, 4, gen.data(), nullptr, 0, nullptr, nullptr) == EC_ERR_ARG);
    CHECK(ec_compile_slp(0, 4, gen.data(), nullptr, 0, nullptr, &prog) == EC_ERR_ARG);
    CHECK(ec_compile_slp(30, 4, gen.data(), nullptr, 0, nullptr, &prog) != EC_OK);
    ec_compile_opts o{};
    o.slot_budget = 33;
    CHECK(ec_compile_slp(10, 4, gen.data(), nullptr, 0, &o, &prog) == EC_ERR_UNSUPPORTED);
    o = ec_compile_opts{};
    o.block_strips = 81;
    CHECK(ec_compile_slp(10, 4, gen.data(), nullptr, 0, &o, &prog) != EC_OK);
    o = ec_compile_opts{};
    o.level = 9;
    CHECK(ec_compile_slp(10, 4, gen.data(), nullptr, 0, &o, &prog) != EC_OK);
    // a singular survivor matrix: data row 0 repeated as parity row 10
    std::vector<uint8_t> sing(gen);
    std::memcpy(&sing[10 * 10], &sing[0], 10);
    const int lose1[] = {1};
    CHECK(ec_compile_slp(10, 4, sing.data(), lose1, 1, nullptr, &prog) == EC_ERR_SINGULAR);
    CHECK(ec_program_query(nullptr, nullptr) == EC_ERR_ARG);
    CHECK(ec_matrix_cauchy(40, 40, gen.data()) != EC_OK);
    for (int s = 0; s <= 9; ++s) CHECK(ec_status_str((ec_status)s) != nullptr);
    ec_program_free(nullptr);
  }
  // the serving loop's output arena: random allocations and releases never
  // overlap, stay in range, keep live + free = size, and coalesce back to
  // one range once everything is released
  {
    const size_t size = 1u << 24, align = 512;
    ec::FirstFit heap(size, align);
    std::vector<std::pair<size_t, size_t>> live;
    uint64_t x = 12345;
    auto rnd = [&x]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    for (int it = 0; it < 4000; ++it) {
      if (!live.empty() && rnd() % 100 < 45) {
        const size_t k = rnd() % live.size();
        heap.release(live[k].first, live[k].second);
        live.erase(live.begin() + (long)k);
      } else {
        size_t got = 0;
        const size_t want = 1 + rnd() % 200000;
        const size_t off = heap.alloc(want, &got);
        if (off != SIZE_MAX) {
          CHECK(got >= want && got % align == 0 && off % align == 0 && off + got <= size);
          live.push_back({off, got});
        }
      }
      std::vector<std::pair<size_t, size_t>> spans(live);
      std::sort(spans.begin(), spans.end());
      for (size_t k = 1; k < spans.size(); ++k) CHECK(spans[k - 1].first + spans[k - 1].second <= spans[k].first);
      size_t total = 0;
      for (auto &sp : spans) total += sp.second;
      for (auto &fr : heap.free_ranges()) total += fr.second;
      CHECK(total == size);
    }
    for (auto &sp : live) heap.release(sp.first, sp.second);
    CHECK(heap.free_ranges().size() == 1 && heap.free_ranges().begin()->second == size);
    size_t got = 0;
    CHECK(heap.alloc(size + 1, &got) == SIZE_MAX);
  }
  // the server's argument checks (made before any HIP call)
  {
    ec_server *sv = nullptr;
    ec_serve_opts o{1u << 20, 2, 4};
    std::vector<uint8_t> host(1 << 16);
    CHECK(ec_server_create(nullptr, 1 << 20, &o, &sv) == EC_ERR_ARG && sv == nullptr);
    CHECK(ec_server_create(host.data(), host.size(), nullptr, &sv) == EC_ERR_ARG);
    CHECK(ec_server_create(host.data(), host.size(), &o, nullptr) == EC_ERR_ARG);
    o.n_slots = 17;
    CHECK(ec_server_create(host.data(), host.size(), &o, &sv) == EC_ERR_ARG);
    o.n_slots = 2;
    o.max_batch = 0;
    CHECK(ec_server_create(host.data(), host.size(), &o, &sv) == EC_ERR_ARG);
    o.max_batch = 4;
    CHECK(ec_server_create(host.data() + 1, host.size() - 1, &o, &sv) == EC_ERR_ALIGN);
    CHECK(ec_server_create(host.data(), 1024, &o, &sv) == EC_ERR_ARG);
    double done = 0;
    CHECK(ec_server_run(nullptr, nullptr, 0, 1, nullptr, nullptr, &done, nullptr, nullptr, nullptr) == EC_ERR_ARG);
    ec_server_free(nullptr);
  }
  std::printf("lib_driver: %d programs compiled and inspected, %d check failures\n", compiled, failures);
  return failures == 0 ? 0 : 1;
}
