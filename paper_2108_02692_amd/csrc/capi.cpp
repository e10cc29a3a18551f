// capi.cpp -- the C ABI of libec (declared in include/ec.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ec.h"
#include "bytecode.hpp"
#include "exec.hpp"
#include "staged.hpp"
#include "gf.hpp"
#include "push.hpp"
#include "slp.hpp"
#include "program.hpp"

using namespace ec;

namespace {

constexpr uint32_t kSlotBudgets[] = {24, 32, 36, 38, 40, 44, 48, 56, 60};  // executor kernels built

// Record overhead of the executor in slot-XOR units: the unfolding trade-off
// of a temporary (one record against the XORs it saves).
constexpr int kRecordCost = 2;

// L2 prefetch distance (strips) of programs compiled with the defaults.
constexpr uint32_t kDefaultPrefetch = 0;

bool supported_slots(uint32_t k) {
  for (uint32_t s : kSlotBudgets)
    if (s == k) return true;
  return false;
}

ec_status make_generator(int n, int p, uint8_t *gen, bool cauchy) {
  if (!gen || n < 1 || p < 0 || n + p > 64) return EC_ERR_ARG;
  const Mat g = cauchy ? cauchy_generator(n, p) : vandermonde_rows_generator(n, p);
  std::memcpy(gen, g.data(), g.size());
  return EC_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Compute units of the current device (queried once per device), or -1.
int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cus;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> g(mu);
  auto it = cus.find(dev);
  if (it != cus.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  cus[dev] = n;
  return n;
}

// Block arguments of a launch: sizes, alignment, and no output overlapping
// an input or another output.
ec_status check_blocks(const uint8_t *const *in, int n_in, uint8_t *const *out, int n_out, size_t block_bytes) {
  if (block_bytes == 0 || block_bytes % 128 != 0) return EC_ERR_ALIGN;
  if (block_bytes / 8 > 0x1FFFFFFFull) return EC_ERR_UNSUPPORTED;  // strip offsets must fit 32 bits
  for (int i = 0; i < n_in; ++i)
    if (!in[i]) return EC_ERR_ARG;
    else if (!aligned16(in[i])) return EC_ERR_ALIGN;
  for (int j = 0; j < n_out; ++j)
    if (!out[j]) return EC_ERR_ARG;
    else if (!aligned16(out[j])) return EC_ERR_ALIGN;
  // outputs must not overlap inputs or each other
  for (int j = 0; j < n_out; ++j) {
    const uintptr_t a = (uintptr_t)out[j];
    for (int i = 0; i < n_in; ++i) {
      const uintptr_t b = (uintptr_t)in[i];
      if (a < b + block_bytes && b < a + block_bytes) return EC_ERR_ARG;
    }
    for (int k = j + 1; k < n_out; ++k) {
      const uintptr_t b = (uintptr_t)out[k];
      if (a < b + block_bytes && b < a + block_bytes) return EC_ERR_ARG;
    }
  }
  return EC_OK;
}

// Block table, strip length, tiles and tile order of a launch.
void set_blocks(ExecArgs &a, const uint8_t *const *in, int n_in, uint8_t *const *out, int n_out,
                size_t block_bytes) {
  for (int i = 0; i < n_in; ++i) a.blk[i] = (uint64_t)(uintptr_t)in[i];
  for (int j = 0; j < n_out; ++j) a.blk[n_in + j] = (uint64_t)(uintptr_t)out[j];
  a.n_in = (uint32_t)n_in;
  a.strip_len = block_bytes / 8;
  a.n_tiles = (uint32_t)((a.strip_len + kTileBytes - 1) / kTileBytes);
  // When the strips lie a multiple of 4 MiB apart, the strips' addresses at
  // one tile offset collide in the memory system's address mapping and
  // waves running side by side on neighbouring tiles slow each other down
  // (measured: 52% of peak at 64 MiB blocks against 60-64% at other sizes);
  // the tiles are then taken from 8 distant segments of the strips, each
  // workgroup's 4 waves on 4 neighbouring tiles of one segment (measured on
  // the data movement alone, 10 x 64 MiB in and 4 x 64 MiB out: 0.735 of
  // peak against 0.728 with consecutive waves in different segments).
  a.seg_shift = 0;
  if (a.strip_len % (4u << 20) == 0 && a.n_tiles % 8 == 0 && (a.n_tiles >> 3) % 4 == 0) a.seg_shift = 3;
  a.seg_mask = (1u << a.seg_shift) - 1;
  a.seg_tiles = a.n_tiles >> a.seg_shift;
}

// LDS of the current device: per workgroup and per compute unit (bytes).
bool device_lds(int *per_group, int *per_cu) {
  static std::mutex mu;
  static std::map<int, std::pair<int, int>> lds;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> g(mu);
  auto it = lds.find(dev);
  if (it == lds.end()) {
    int a = 0, b = 0;
    if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
      return false;
    it = lds.emplace(dev, std::make_pair(a, b)).first;
  }
  *per_group = it->second.first;
  *per_cu = it->second.second;
  return true;
}

// A staged launch: one workgroup per tile at a time, its waves on the stage
// parts; as many workgroups as the LDS (8 KiB per input block each) and the
// registers let stay resident, each looping over tiles.
ec_status launch_staged(const ec_program *prog, ExecArgs &a, int n_cus, ec_stream stream) {
  const uint64_t lds_bytes = (uint64_t)a.n_in * kStageBytesPerBlock;
  int per_group = 0, per_cu = 0;
  if (!device_lds(&per_group, &per_cu)) return EC_ERR_DEVICE;
  if (lds_bytes > (uint64_t)per_group || lds_bytes > (uint64_t)per_cu) return EC_ERR_UNSUPPORTED;
  a.n_parts = (uint32_t)prog->stage_part_off.size();
  for (uint32_t q = 0; q < a.n_parts; ++q) a.part_off[q] = prog->stage_part_off[q];
  const uint64_t groups_per_cu =
      std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)per_cu / lds_bytes, (uint64_t)waves_per_simd(prog->slots)));
  const int grid = (int)std::min<uint64_t>(a.n_tiles, (uint64_t)n_cus * groups_per_cu);
  if (staged_launch(prog->slots, a, grid, (uint32_t)lds_bytes, (hipStream_t)stream) != 0) return EC_ERR_DEVICE;
  return EC_OK;
}

// Native kernel `which` (0: the whole program, one wave per tile; 1: the
// pair parts and 2: the block parts, one wave per (tile, part)): as many
// workgroups as stay resident, each looping over its work items.
ec_status launch_native(ec_program *prog, int which, const ExecArgs &a, int n_cus, ec_stream stream) {
  int dev = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return EC_ERR_DEVICE;
  ec_status st = EC_OK;
  hipFunction_t fn = prog->native_function(dev, which, &per_cu, &st);
  if (!fn) return st;
  ec::NativeArgs na{};
  for (int b = 0; b < kMaxBlocks; ++b) na.blk[b] = a.blk[b];
  na.sl = (uint32_t)a.strip_len;
  na.n_tiles = a.n_tiles;
  na.seg_shift = a.seg_shift;
  na.seg_mask = a.seg_mask;
  na.seg_tiles = a.seg_tiles;
  na.n_parts = which == 1 ? (uint32_t)prog->pair_parts.size() : which == 2 ? (uint32_t)prog->parts.size() : 1u;
  const uint64_t n_work = (uint64_t)a.n_tiles * na.n_parts;
  const int grid = (int)std::min<uint64_t>((n_work + 3) / 4, (uint64_t)n_cus * per_cu);
  return ec::native_launch(fn, na, grid, (hipStream_t)stream) == 0 ? EC_OK : EC_ERR_DEVICE;
}

ec_status launch(const ec_program *prog, const uint8_t *const *in, uint8_t *const *out, size_t block_bytes,
                 ec_stream stream) {
  if (!prog || !in || !out) return EC_ERR_ARG;
  const int n_in = (int)prog->in_blocks.size(), n_out = (int)prog->out_blocks.size();
  ec_status st = check_blocks(in, n_in, out, n_out, block_bytes);
  if (st != EC_OK) return st;
  const uint32_t *words = const_cast<ec_program *>(prog)->device_words(&st);
  if (!words) return st;
  ExecArgs a{};
  set_blocks(a, in, n_in, out, n_out, block_bytes);
  a.prog = words;
  const int n_cus = device_cus();
  if (n_cus <= 0) return EC_ERR_DEVICE;
  if (prog->split == EC_SPLIT_STAGED) return launch_staged(prog, a, n_cus, stream);
  const uint64_t resident = (uint64_t)n_cus * waves_per_simd(prog->slots);  // workgroups of 4 waves
  // Row split for short stripes: single-row parts first, else pairs of
  // rows, else parts of whole output blocks.  Measured on RS(10,4) encodes
  // (32 row parts, 16 pair parts or 4 block parts against one wave per
  // tile): 8 KiB - 256 KiB blocks 10.5 - 10.8 us with row parts, 20.2 - 20.7
  // us with block parts, 28.5 - 30.3 us unsplit; 1 MiB 18.0 us with pair
  // parts, 20.9 us with block parts, 23.7 us with row parts; 8 MiB 47 us
  // with block parts forced against 32 us unsplit: every part reads its
  // inputs, so once the waves are busy anyway a split only adds work.
  a.n_parts = 1;
  a.part_off[0] = 0;
  const uint64_t waves = 4 * resident;
  const std::vector<uint32_t> *off = nullptr;
  const uint64_t nb = prog->parts.size(), nr = prog->row_parts.size(), np = prog->pair_parts.size();
  const uint64_t ns = prog->pass_parts.size();
  if (prog->split == EC_SPLIT_ROWS) {
    if (nr) off = &prog->row_part_off;
  } else if (prog->split == EC_SPLIT_PAIRS) {
    if (np) off = &prog->pair_part_off;
  } else if (prog->split == EC_SPLIT_ALWAYS) {
    if (nb) off = &prog->part_off;
  } else if (prog->split == EC_SPLIT_PASSES) {
    if (ns) off = &prog->pass_part_off;
  } else if (prog->split == EC_SPLIT_AUTO) {
    const uint64_t fine = 2ull * 4 * (uint64_t)n_cus;
    const bool nat_whole = !prog->native_code[0].empty(), nat_pairs = !prog->native_code[1].empty();
    const bool nat_blocks = !prog->native_code[2].empty() && nb;
    if (nat_pairs && np && a.n_tiles * np <= (nat_blocks ? fine / 4 : fine / 2)) {
      // With native kernels: pair parts while there is at most half a wave
      // per SIMD (one without block parts), then block parts up to one wave
      // per SIMD, else the whole program.  Measured on RS(10,4) encodes and
      // decodes of {2,4,5,6} (plain / compressed): 16 - 256 KiB blocks 6.6 -
      // 9.2 us with native pair parts or block parts alike (11 - 15 us with
      // the interpreter's row parts); 512 KiB 9.0 - 9.3 us with block parts
      // against 9.7 - 9.8 us with pairs; 1 MiB 9.5 - 9.7 us with block parts
      // against 13.4 - 15.8 us whole and 15.2 - 15.5 us in pairs; 2 MiB
      // 10.2 - 10.5 us against 13.9 - 17.4 us whole; 4 MiB 15.0 / 19.1 us
      // whole against 18.8 / 18.8 us in block parts.
      off = &prog->pair_part_off;
    } else if (nat_blocks && a.n_tiles * nb <= fine / 2) {
      off = &prog->part_off;
    } else if (nat_whole) {
      off = nullptr;
    } else if (nr && a.n_tiles * nr <= fine) {
      // The finest set that fits: row or pair parts while there are at most
      // two waves per SIMD (their chains run side by side), block parts
      // while all their waves are resident; else pass parts when the
      // program needs several passes over the inputs.
      off = &prog->row_part_off;
    } else if (np && a.n_tiles * np <= fine) {
      off = &prog->pair_part_off;
    } else if (nb && a.n_tiles * nb <= waves) {
      off = &prog->part_off;
    } else if (ns) {
      off = &prog->pass_part_off;
    }
  }
  if (off) {
    a.n_parts = (uint32_t)off->size();
    for (uint32_t q = 0; q < a.n_parts; ++q) a.part_off[q] = (*off)[q];
  }
  // native kernels, where the program has one for the launch's split
  if (off == &prog->pair_part_off && !prog->native_code[1].empty())
    return launch_native(const_cast<ec_program *>(prog), 1, a, n_cus, stream);
  if (off == &prog->part_off && !prog->native_code[2].empty())
    return launch_native(const_cast<ec_program *>(prog), 2, a, n_cus, stream);
  if (!off && !prog->native_code[0].empty()) return launch_native(const_cast<ec_program *>(prog), 0, a, n_cus, stream);
  // As many workgroups as stay resident (4 waves each, one per SIMD, times
  // the waves per SIMD the slot budget allows), each looping over its work
  // items: measured 3-6% faster than one workgroup per 4 tiles.
  const uint64_t n_work = (uint64_t)a.n_tiles * a.n_parts;
  const int grid = (int)std::min<uint64_t>((n_work + 3) / 4, resident);
  if (exec_launch(prog->slots, a, grid, (hipStream_t)stream) != 0) return EC_ERR_DEVICE;
  return EC_OK;
}

void export_stage(const Slp &s, std::vector<int32_t> &v) {
  auto term = [](int t) -> int32_t {
    if (t == kZero) return -1;
    if (is_const(t)) return -(t - kConstBase) - 2;
    return t;
  };
  v.push_back((int32_t)s.stmts.size());
  v.push_back((int32_t)s.outputs.size());
  for (const Stmt &st : s.stmts) {
    v.push_back(st.var);
    v.push_back((int32_t)st.ops.size());
    for (int o : st.ops) v.push_back(term(o));
  }
  for (int o : s.outputs) v.push_back(term(o));
}

}  // namespace

extern "C" {

ec_status ec_matrix_cauchy(int n, int p, uint8_t *gen) { return make_generator(n, p, gen, true); }
ec_status ec_matrix_vandermonde(int n, int p, uint8_t *gen) { return make_generator(n, p, gen, false); }

ec_status ec_compile_slp(int n, int p, const uint8_t *gen, const int *erased, int n_erased,
                         const ec_compile_opts *opts, ec_program **out) {
  if (!out) return EC_ERR_ARG;
  *out = nullptr;
  if (!gen || n < 1 || p < 0 || n + p > kMaxBlocks || n_erased < 0) return EC_ERR_ARG;
  if (n_erased > 0 && !erased) return EC_ERR_ARG;
  if (n_erased > p) return EC_ERR_TOO_MANY_ERASURES;
  for (int i = 0; i < n_erased; ++i) {
    if (erased[i] < 0 || erased[i] >= n + p) return EC_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (erased[j] == erased[i]) return EC_ERR_ARG;
  }
  ec_compile_opts o{EC_LEVEL_CO_FU_SCHED, 0, EC_COMPRESS_XORREPAIR, 0, kDefaultPrefetch, EC_SPLIT_AUTO,
                    EC_SCHED_PUSH, 0};
  if (opts) o = *opts;
  if (o.level > EC_LEVEL_CO_FU_SCHED || o.compress > EC_COMPRESS_REPAIR) return EC_ERR_UNSUPPORTED;
  if (o.scheduler > EC_SCHED_GREEDY) return EC_ERR_UNSUPPORTED;
  if (o.native > (EC_NATIVE_WHOLE | EC_NATIVE_PAIRS | EC_NATIVE_BLOCKS) || (o.native && o.split == EC_SPLIT_STAGED))
    return EC_ERR_UNSUPPORTED;
  if (o.slot_budget != 0 && !supported_slots(o.slot_budget)) return EC_ERR_UNSUPPORTED;
  if (o.block_strips > (uint32_t)(8 * n) || o.prefetch > 64) return EC_ERR_ARG;
  if (o.split > EC_SPLIT_STAGED) return EC_ERR_UNSUPPORTED;
  if (o.split == EC_SPLIT_STAGED && (uint64_t)n * kStageBytesPerBlock > kMaxStageBytes)
    return EC_ERR_UNSUPPORTED;

  std::unique_ptr<ec_program> prog(new (std::nothrow) ec_program);
  if (!prog) return EC_ERR_NOMEM;
  prog->n = n;
  prog->p = p;
  prog->decode = n_erased > 0;
  prog->level = (int)o.level;
  const Mat g(gen, gen + (size_t)(n + p) * n);
  Mat rows;
  if (!prog->decode) {
    rows.assign(g.begin() + (size_t)n * n, g.end());
    for (int i = 0; i < n; ++i) prog->in_blocks.push_back(i);
    for (int j = 0; j < p; ++j) prog->out_blocks.push_back(n + j);
  } else {
    std::vector<int> er(erased, erased + n_erased);
    if (decode_rows(n, p, g, er, rows, prog->in_blocks) != 0) return EC_ERR_SINGULAR;
    prog->out_blocks = er;
  }
  const int n_in = (int)prog->in_blocks.size(), n_out = (int)prog->out_blocks.size();
  const std::vector<Bits> brows = bitmatrix_rows(n_out, n, rows);
  const int n_const = 8 * n;

  // The paper's whole-matrix pipeline (Secs. 2-6) is built on first export
  // only (it is for inspection; the executed program is built below).
  prog->plain = plain_slp(brows, n_const);
  prog->brows = brows;
  prog->rebuild = o.compress == EC_COMPRESS_XORREPAIR;

  // The executed program, in push form.
  const int width = o.block_strips ? (int)o.block_strips : 8;
  const bool greedy = o.scheduler == EC_SCHED_GREEDY;
  // The strip order: the push orderer at level CO_FU_SCHED, made once per
  // program; or the bottom-up greedy heuristic of Sec. 6.6 with the slot
  // budget k as its cache (within column blocks when there are
  // temporaries), made for each budget tried.
  auto order = [&](PushDag &dg, int k) {
    if (greedy) push_order_greedy(dg, o.level >= EC_LEVEL_CO ? width : 0, k);
  };
  auto push_ordered = [&](PushDag &dg) {
    if (!greedy && o.level >= EC_LEVEL_CO_FU_SCHED) push_order(dg, width);
  };
  PushDag dag;
  if (o.level == EC_LEVEL_PLAIN) {
    dag = push_plain(brows, n_const);
  } else {
    dag = push_blocked(brows, n_const, width, o.compress == EC_COMPRESS_XORREPAIR, o.level >= EC_LEVEL_CO_FU);
    if (o.level >= EC_LEVEL_CO_FU_SCHED) {
      push_unfold(dag, kRecordCost);
      push_ordered(dag);
    }
  }
  PushOpts po;
  po.prefetch = (int)o.prefetch;
  auto place = [&]() -> int {
    if (o.slot_budget) {
      po.slots = (int)o.slot_budget;
      order(dag, po.slots);
      return push_schedule(dag, n_in, po, prog->code);
    }
    // The budgets that set the executor's occupancy (4, 3 and 2 waves per
    // SIMD for 24, 38 and 48 slots; 32 and 44 in between), smallest first:
    // the first that holds every row in one pass over the inputs with a ring
    // of at least 3 loads.  Past 48, only to save a pass: 56 and 60 slots
    // still run 2 waves per SIMD (up to 256 VGPRs), and rows that need a
    // second pass would read every input again.
    int rc = -1;
    for (uint32_t k : {24u, 32u, 38u, 44u, 48u}) {
      po.slots = (int)k;
      order(dag, po.slots);
      rc = push_schedule(dag, n_in, po, prog->code);
      if (rc == 0 && ((prog->code.passes == 1 && prog->code.ring >= 3) || k == 48)) break;
    }
    if (rc != 0 || prog->code.passes > 1) {
      PushOpts wide = po;
      for (int k : {56, 60}) {
        wide.slots = k;
        PushDag trial = dag;
        order(trial, k);
        PushCode code;
        if (push_schedule(trial, n_in, wide, code) == 0 && code.passes == 1 && code.ring >= 3) {
          dag = trial;
          prog->code = code;
          po = wide;
          return 0;
        }
      }
      po.slots = 48;  // (the order for 48 stays in dag: order() was last applied with 48)
    }
    return rc;
  };
  int rc = place();
  // By default, a few more unfolded temporaries are worth it when they let
  // the program run at 3 waves per SIMD (38 slots) instead of 2.
  if (rc == 0 && !o.slot_budget && po.slots > 38 && o.level >= EC_LEVEL_CO_FU_SCHED && n_out * 8 <= 32) {
    for (int cost : {3, 4, 6}) {
      PushDag trial = dag;
      push_unfold(trial, cost);
      push_ordered(trial);
      order(trial, 38);
      PushCode code;
      PushOpts p38 = po;
      p38.slots = 38;
      if (push_schedule(trial, n_in, p38, code) == 0 && code.passes == 1 && code.ring >= 3) {
        dag = trial;
        prog->code = code;
        po = p38;
        break;
      }
    }
  }
  // Too many temporaries open for the budget: unfold more of them (in the
  // limit every temporary is inlined and none is open) until it fits.
  for (int cost : {4, 8, 16, 64, 1 << 20}) {
    if (rc == 0 || o.level == EC_LEVEL_PLAIN) break;
    push_unfold(dag, cost);
    push_ordered(dag);
    rc = place();
  }
  if (rc != 0) return EC_ERR_CAPACITY;
  {
    const std::vector<Bits> val = push_eval(dag);
    for (size_t r = 0; r < brows.size(); ++r)
      if (!(val[r] == brows[r])) return EC_ERR_UNSUPPORTED;
  }
  prog->exec = push_as_slp(dag);
  prog->slots = po.slots;
  if (!simulate_code(prog->code.words, prog->slots, n_in, n_out, brows)) return EC_ERR_UNSUPPORTED;

  // Row-split parts at two granularities, each part scheduled alone on the
  // same slot budget (so with a deeper load ring) and checked like the whole
  // program; a set is dropped if any of its parts does not fit in one pass:
  //  * groups of whole output blocks (at most kMaxParts): mid-size stripes
  //    and batches;
  //  * single bit rows, or runs of floor or ceil(rows / kMaxRowParts) rows
  //    beyond 4 output blocks (at most kMaxRowParts): the shortest stripes,
  //    where a wave's time is its chain of records and a single row needs
  //    only about half the inputs;
  //  * pairs of rows, or runs of pairs beyond 4 output blocks (at most
  //    kMaxRowParts / 2): stripes a little too long for single rows.
  // Parts run where a lone wave's chain of records is the time, and there
  // the plain rows win whatever the level: one record per input strip and
  // no records for temporaries (measured on RS(10,4) encodes, 8 KiB - 1 MiB
  // blocks: row parts 10.5-10.8 us plain against 11.8-12.1 us compressed,
  // block parts 20.2-20.7 against 22.3-22.9 us; 2-20% on every codec tried).
  PushDag pdag = o.level == EC_LEVEL_PLAIN ? dag : push_plain(brows, n_const);
  if (greedy && o.level != EC_LEVEL_PLAIN) push_order_greedy(pdag, 0, po.slots);
  prog->split = (int)o.split;
  prog->image = prog->code.words;
  prog->part_off.clear();
  prog->row_part_off.clear();
  prog->pair_part_off.clear();
  const int n_rows = 8 * n_out;
  // Groups of whole units of `unit` rows; consecutive groups differ by at
  // most one unit and together cover every row.
  auto build_parts = [&](int unit, int max_groups, std::vector<PushCode> &set) -> bool {
    const int units = n_rows / unit;
    if (units * unit != n_rows) return false;
    const int groups = std::min(units, max_groups);
    for (int g = 0; g < groups; ++g) {
      PushOpts pp = po;
      pp.row_lo = unit * (g * units / groups);
      pp.row_hi = unit * ((g + 1) * units / groups);
      pp.max_ring = 24;
      PushCode part;
      if (push_schedule(pdag, n_in, pp, part) != 0 || part.passes != 1) {
        set.clear();
        return true;
      }
      if (!simulate_code(part.words, prog->slots, n_in, n_out, brows, pp.row_lo, pp.row_hi)) return false;
      set.push_back(std::move(part));
    }
    return true;
  };
  const bool split_parts = o.split != EC_SPLIT_NEVER && o.split != EC_SPLIT_STAGED;
  if (split_parts) {
    if (n_out > 1 && !build_parts(8, kMaxParts, prog->parts)) return EC_ERR_UNSUPPORTED;
    if (n_rows > 1 && !build_parts(1, kMaxRowParts, prog->row_parts)) return EC_ERR_UNSUPPORTED;
    if (n_rows > 2 && !build_parts(2, kMaxRowParts / 2, prog->pair_parts)) return EC_ERR_UNSUPPORTED;
  }
  // Pass parts: when the rows need several passes over the inputs, the
  // fewest groups of whole output blocks that each fit one pass, scheduled
  // from the program itself (its level and order).  The parts of one tile
  // run on neighbouring waves of one workgroup at the same time, so an
  // input strip-tile is fetched from HBM once and found in the caches by the
  // other parts, where a single wave would read it again from HBM on every
  // pass (the register file holds one level of the cache hierarchy, the
  // caches the next).
  prog->pass_parts.clear();
  prog->pass_part_off.clear();
  if (split_parts && prog->code.passes > 1) {
    for (int groups = prog->code.passes; groups <= std::min(n_out, kMaxParts); ++groups) {
      std::vector<PushCode> set;
      bool fits = true;
      for (int g = 0; g < groups && fits; ++g) {
        PushOpts pp = po;
        pp.row_lo = 8 * (g * n_out / groups);
        pp.row_hi = 8 * ((g + 1) * n_out / groups);
        PushCode part;
        fits = push_schedule(dag, n_in, pp, part) == 0 && part.passes == 1;
        if (fits) {
          if (!simulate_code(part.words, prog->slots, n_in, n_out, brows, pp.row_lo, pp.row_hi))
            return EC_ERR_UNSUPPORTED;
          set.push_back(std::move(part));
        }
      }
      if (fits) {
        prog->pass_parts = std::move(set);
        break;
      }
    }
  }
  // Stage parts: min(4, rows) runs of consecutive rows, one per wave of a
  // staged workgroup, scheduled from the program itself on its budget.
  // Their strip loads read LDS, so a part may take several passes (each
  // re-reads the staged strips, not HBM) and no prefetch records are made.
  prog->stage_parts.clear();
  prog->stage_part_off.clear();
  if (o.split == EC_SPLIT_STAGED) {
    const int groups = std::min(kStageWaves, n_rows);
    for (int g = 0; g < groups; ++g) {
      PushOpts pp = po;
      pp.prefetch = 0;
      pp.row_lo = g * n_rows / groups;
      pp.row_hi = (g + 1) * n_rows / groups;
      PushCode part;
      if (push_schedule(dag, n_in, pp, part) != 0) return EC_ERR_CAPACITY;
      if (!simulate_code(part.words, prog->slots, n_in, n_out, brows, pp.row_lo, pp.row_hi))
        return EC_ERR_UNSUPPORTED;
      prog->stage_parts.push_back(std::move(part));
    }
  }
  for (const PushCode &part : prog->parts) {
    prog->part_off.push_back((uint32_t)prog->image.size());
    prog->image.insert(prog->image.end(), part.words.begin(), part.words.end());
  }
  for (const PushCode &part : prog->row_parts) {
    prog->row_part_off.push_back((uint32_t)prog->image.size());
    prog->image.insert(prog->image.end(), part.words.begin(), part.words.end());
  }
  for (const PushCode &part : prog->pair_parts) {
    prog->pair_part_off.push_back((uint32_t)prog->image.size());
    prog->image.insert(prog->image.end(), part.words.begin(), part.words.end());
  }
  for (const PushCode &part : prog->pass_parts) {
    prog->pass_part_off.push_back((uint32_t)prog->image.size());
    prog->image.insert(prog->image.end(), part.words.begin(), part.words.end());
  }
  for (const PushCode &part : prog->stage_parts) {
    prog->stage_part_off.push_back((uint32_t)prog->image.size());
    prog->image.insert(prog->image.end(), part.words.begin(), part.words.end());
  }

  // Native kernels: the whole program's records, and the pair parts' and
  // block parts' (when the program has them), as straight-line code.
  for (int which = 0; which < ec::kNativeKernels; ++which) {
    if (!(o.native & (1u << which))) continue;
    std::vector<std::vector<uint32_t>> parts;
    if (which == 0) {
      parts.push_back(prog->code.words);
    } else {
      for (const PushCode &part : which == 1 ? prog->pair_parts : prog->parts) parts.push_back(part.words);
    }
    if (parts.empty()) continue;
    std::string log;
    prog->native_src[which] = ec::native_source(parts, prog->slots, n_in + n_out);
    const ec_status st = ec::native_compile(prog->native_src[which], &prog->native_code[which], &log);
    if (st != EC_OK) return st;
  }

  ec_program_info &info = prog->info;
  info.n = (uint32_t)n;
  info.p = (uint32_t)p;
  info.n_in = (uint32_t)prog->in_blocks.size();
  info.n_out = (uint32_t)n_out;
  const Slp &f = prog->exec;
  info.n_stmt = (uint32_t)f.stmts.size();
  info.n_xor2 = (uint32_t)count_xor(f);
  info.n_mem = (uint32_t)count_mem(f);
  info.nvar = (uint32_t)f.stmts.size();
  info.plain_xor2 = (uint32_t)count_xor(prog->plain);
  info.slots = (uint32_t)prog->slots;
  info.peak_open = (uint32_t)prog->code.peak_open;
  info.ring = (uint32_t)prog->code.ring;
  info.passes = (uint32_t)prog->code.passes;
  info.n_loads = (uint32_t)prog->code.n_loads;
  info.n_stores = (uint32_t)prog->code.n_stores;
  info.n_records = (uint32_t)prog->code.n_records;
  info.n_ops = (uint32_t)prog->code.n_ops;
  info.n_words = (uint32_t)prog->code.words.size();
  info.n_parts = (uint32_t)prog->parts.size();
  info.n_row_parts = (uint32_t)prog->row_parts.size();
  info.n_pair_parts = (uint32_t)prog->pair_parts.size();
  info.n_pass_parts = (uint32_t)prog->pass_parts.size();
  info.scheduler = o.scheduler;
  info.n_stage_parts = (uint32_t)prog->stage_parts.size();
  info.native = 0;
  for (int which = 0; which < ec::kNativeKernels; ++which)
    if (!prog->native_code[which].empty()) info.native |= 1u << which;
  info.in_blocks = prog->in_blocks.data();
  info.out_blocks = prog->out_blocks.data();
  *out = prog.release();
  return EC_OK;
}

ec_status ec_program_query(const ec_program *prog, ec_program_info *out) {
  if (!prog || !out) return EC_ERR_ARG;
  *out = prog->info;
  return EC_OK;
}

ec_status ec_encode(const ec_program *prog, const uint8_t *const *data, uint8_t *const *parity,
                    size_t block_bytes, ec_stream stream) {
  if (!prog || prog->decode) return EC_ERR_ARG;
  return launch(prog, data, parity, block_bytes, stream);
}

ec_status ec_decode(const ec_program *prog, const uint8_t *const *survivors, uint8_t *const *recovered,
                    size_t block_bytes, ec_stream stream) {
  if (!prog || !prog->decode) return EC_ERR_ARG;
  return launch(prog, survivors, recovered, block_bytes, stream);
}

void ec_program_free(ec_program *prog) { delete prog; }

const char *ec_status_str(ec_status s) {
  switch (s) {
    case EC_OK: return "ok";
    case EC_ERR_ARG: return "invalid argument";
    case EC_ERR_ALIGN: return "block size not a multiple of 128 or pointer not 16-byte aligned";
    case EC_ERR_TOO_MANY_ERASURES: return "more erasures than parity blocks";
    case EC_ERR_SINGULAR: return "survivor matrix is singular";
    case EC_ERR_NOMEM: return "out of memory";
    case EC_ERR_DEVICE: return "HIP device error";
    case EC_ERR_UNSUPPORTED: return "unsupported option or size";
    case EC_ERR_CAPACITY: return "program exceeds the register slot budget";
  }
  return "unknown status";
}

ec_status ec_program_export(const ec_program *prog, int stage, int32_t *buf, size_t cap, size_t *len) {
  if (!prog || !len) return EC_ERR_ARG;
  const Slp *s = nullptr;
  if (stage >= EC_STAGE_CO && stage <= EC_STAGE_SCHED) const_cast<ec_program *>(prog)->paper_stages();
  switch (stage) {
    case EC_STAGE_PLAIN: s = &prog->plain; break;
    case EC_STAGE_CO: s = prog->level >= EC_LEVEL_CO ? &prog->co : nullptr; break;
    case EC_STAGE_FU: s = prog->level >= EC_LEVEL_CO_FU ? &prog->fu : nullptr; break;
    case EC_STAGE_SCHED: s = prog->level >= EC_LEVEL_CO_FU_SCHED ? &prog->sched : nullptr; break;
    case EC_STAGE_EXEC: s = &prog->exec; break;
    default: break;
  }
  if (!s) return EC_ERR_ARG;
  std::vector<int32_t> v;
  export_stage(*s, v);
  *len = v.size();
  if (buf) std::memcpy(buf, v.data(), std::min(cap, v.size()) * sizeof(int32_t));
  return EC_OK;
}

ec_status ec_program_export_greedy(const ec_program *prog, int capacity, int32_t *buf, size_t cap, size_t *len) {
  if (!prog || !len || capacity < 1 || prog->level < EC_LEVEL_CO_FU) return EC_ERR_ARG;
  const_cast<ec_program *>(prog)->paper_stages();
  std::vector<int32_t> v;
  try {
    export_stage(greedy_schedule(prog->fu, capacity), v);
  } catch (const std::bad_alloc &) {
    return EC_ERR_NOMEM;
  }
  *len = v.size();
  if (buf) std::memcpy(buf, v.data(), std::min(cap, v.size()) * sizeof(int32_t));
  return EC_OK;
}

ec_status ec_device_copy(void *dst, const void *src, size_t bytes, ec_stream stream) {
  if (!dst || !src || bytes == 0) return EC_ERR_ARG;
  if (bytes % 16 || !aligned16(dst) || !aligned16(src)) return EC_ERR_ALIGN;
  const uintptr_t a = (uintptr_t)dst, b = (uintptr_t)src;
  if (a < b + bytes && b < a + bytes) return EC_ERR_ARG;
  const int n_cus = device_cus();
  if (n_cus <= 0) return EC_ERR_DEVICE;
  return copy_launch(src, dst, bytes, n_cus, (hipStream_t)stream) == 0 ? EC_OK : EC_ERR_DEVICE;
}

ec_status ec_stripe_stream(const uint8_t *const *in, int n_in, uint8_t *const *out, int n_out, size_t block_bytes,
                           ec_stream stream) {
  if (!in || !out || n_in < 1 || n_out < 0 || n_in + n_out > kMaxBlocks) return EC_ERR_ARG;
  ec_status st = check_blocks(in, n_in, out, n_out, block_bytes);
  if (st != EC_OK) return st;
  ExecArgs a{};
  set_blocks(a, in, n_in, out, n_out, block_bytes);
  const int n_cus = device_cus();
  if (n_cus <= 0) return EC_ERR_DEVICE;
  // 3 waves per SIMD: measured on the 10 x 64 MiB + 4 x 64 MiB movement
  // 0.749 of peak at 2 or 3, 0.741 at 4, 0.735 at 8 (with the strips
  // loaded 8 at a time; 16 or more at a time did no better)
  const int grid = (int)std::min<uint64_t>(((uint64_t)a.n_tiles + 3) / 4, (uint64_t)n_cus * 3);
  return stream_launch(a, (uint32_t)n_out, grid, (hipStream_t)stream) == 0 ? EC_OK : EC_ERR_DEVICE;
}

ec_status ec_program_upload(ec_program *prog) {
  if (!prog) return EC_ERR_ARG;
  ec_status st = EC_OK;
  if (!prog->device_words(&st)) return st;
  for (int which = 0; which < ec::kNativeKernels; ++which)
    if (!prog->native_code[which].empty()) {
      int dev = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess) return EC_ERR_DEVICE;
      if (!prog->native_function(dev, which, &per_cu, &st)) return st;
    }
  return EC_OK;
}

ec_status ec_program_native_source(const ec_program *prog, int kernel, const char **src, size_t *len) {
  if (!prog || !src || !len) return EC_ERR_ARG;
  const int which = kernel == EC_NATIVE_WHOLE ? 0 : kernel == EC_NATIVE_PAIRS ? 1 : kernel == EC_NATIVE_BLOCKS ? 2 : -1;
  if (which < 0) return EC_ERR_ARG;
  const std::string &s = prog->native_src[which];
  if (s.empty()) return EC_ERR_ARG;
  *src = s.c_str();
  *len = s.size();
  return EC_OK;
}

ec_status ec_program_upload_many(ec_program *const *progs, int n) {
  if (n < 0 || (n > 0 && !progs)) return EC_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!progs[i]) return EC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return EC_ERR_DEVICE;
  std::vector<const std::vector<uint32_t> *> need;
  for (int i = 0; i < n; ++i)
    if (!progs[i]->device_words_present(dev)) need.push_back(&progs[i]->image);
  if (need.empty()) return EC_OK;
  const size_t bytes = ec::pool_missing_bytes(dev, need);
  if (bytes) {
    const ec_status st = ec::pool_reserve(dev, bytes);
    if (st != EC_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    ec_status st = EC_OK;
    if (!progs[i]->device_words(dev, &st)) return st;
    int per_cu = 0;
    for (int which = 0; which < ec::kNativeKernels; ++which)
      if (!progs[i]->native_code[which].empty() && !progs[i]->native_function(dev, which, &per_cu, &st)) return st;
  }
  return EC_OK;
}

ec_status ec_program_pool_stats(int *chunks, int *images, size_t *bytes_used) {
  if (!chunks && !images && !bytes_used) return EC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return EC_ERR_DEVICE;
  ec::pool_stats(dev, chunks, images, bytes_used);
  return EC_OK;
}

ec_status ec_program_part_bytecode(const ec_program *prog, int part, const uint32_t **words, size_t *n_words) {
  if (!prog || !words || !n_words || part < 0) return EC_ERR_ARG;
  const int nb = (int)prog->parts.size();
  const int nr = (int)prog->row_parts.size();
  const int np = (int)prog->pair_parts.size();
  const int ns = (int)prog->pass_parts.size();
  if (part >= nb + nr + np + ns + (int)prog->stage_parts.size()) return EC_ERR_ARG;
  const PushCode &c = part < nb             ? prog->parts[part]
                      : part < nb + nr      ? prog->row_parts[part - nb]
                      : part < nb + nr + np ? prog->pair_parts[part - nb - nr]
                      : part < nb + nr + np + ns ? prog->pass_parts[part - nb - nr - np]
                                                 : prog->stage_parts[part - nb - nr - np - ns];
  *words = c.words.data();
  *n_words = c.words.size();
  return EC_OK;
}

ec_status ec_program_bytecode(const ec_program *prog, const uint32_t **words, size_t *n_words) {
  if (!prog || !words || !n_words) return EC_ERR_ARG;
  *words = prog->code.words.data();
  *n_words = prog->code.words.size();
  return EC_OK;
}

}  // extern "C"
