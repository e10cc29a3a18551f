// native.cpp -- straight-line kernels of compiled programs (native.hpp).
#include "native.hpp"

#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <utility>

#include "bytecode.hpp"
#include "exec.hpp"

namespace ec {

namespace {

// The register slots v[4 : 4+4K) as pinned groups of 32, 16 and 8 VGPRs
// (the accumulator is v[0:3]), as the interpreter pins them.
std::vector<std::pair<int, int>> slot_groups(int K) {
  std::vector<std::pair<int, int>> out;
  int lo = 4, left = 4 * K;
  for (int size : {32, 16, 8})
    while (left >= size) {
      out.push_back({lo, size});
      lo += size;
      left -= size;
    }
  return out;
}

std::string fmt(const char *f, int a = 0, int b = 0, int c = 0, int d = 0) {
  char buf[160];
  std::snprintf(buf, sizeof buf, f, a, b, c, d);
  return buf;
}

// One asm line inside the C string of the kernel's asm statement.
void line(std::string &s, const std::string &ins) { s += "        \"" + ins + "\\n\\t\"\n"; }

// The records as instructions, in record order (so the memory operations
// keep their order and the records' exact vmcnt waits hold):
//   WAIT    s_waitcnt vmcnt(n)
//   PULL    acc = slot (4 v_mov)
//   LD      global_load_dwordx4 slot, strip offset, block base, non-temporal
//   STORE   global_store_dwordx4 acc, non-temporal, then one wait state
//           before the next VALU may overwrite acc
//   run     slot ^= acc (4 v_xor) per operand
// PREFETCH records are hints and are left out (each wait then counts one
// memory operation fewer in flight than it allows: it waits no less).
std::string body(const std::vector<uint32_t> &w) {
  std::string s;
  size_t pc = 0;
  while (pc + 1 < w.size()) {
    const uint32_t h0 = w[pc], h1 = w[pc + 1];
    const uint32_t kind = bc::h0_kind(h0);
    if (kind == bc::HALT) break;
    const int n = (int)(bc::h0_bytes(h0) - 8) / 4;
    const int pull = (int)bc::h0_pull(h0), wait = (int)bc::h1_wait(h1), ld = (int)bc::h1_ld(h1);
    const int blk = (int)bc::h1_blk(h1), j = (int)bc::h1_j(h1);
    if (kind == bc::INPUT || kind == bc::INPUT_LD) line(s, fmt("s_waitcnt vmcnt(%d)", wait));
    if (kind == bc::INPUT || kind == bc::INPUT_LD || kind == bc::VALUE || kind == bc::STORE)
      for (int q = 0; q < 4; ++q) line(s, fmt("v_mov_b32 v%d, v%d", q, 4 + 4 * pull + q));
    if (kind == bc::INPUT_LD || kind == bc::LOAD)
      line(s, fmt("global_load_dwordx4 v[%d:%d], %%[o%d], %%[b%d] nt", 4 + 4 * ld, 7 + 4 * ld, j, blk));
    if (kind == bc::STORE) {
      line(s, fmt("global_store_dwordx4 %%[o%d], v[0:3], %%[b%d] nt", j, blk));
      line(s, "s_nop 1");
    }
    for (int i = 0; i < n; ++i) {
      const int slot = (int)(w[pc + 2 + i] / 4);
      for (int q = 0; q < 4; ++q) line(s, fmt("v_xor_b32 v%d, v%d, v%d", 4 + 4 * slot + q, 4 + 4 * slot + q, q));
    }
    pc += bc::h0_bytes(h0) / 4;
  }
  return s;
}

const char *kHead = R"(// Generated from a compiled XOR program: one asm statement per tile holds
// the program's loads, XORs and stores in record order.
typedef unsigned int uint32_t;
typedef unsigned long long uint64_t;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v8u __attribute__((ext_vector_type(8)));
typedef uint32_t v16u __attribute__((ext_vector_type(16)));
typedef uint32_t v32u __attribute__((ext_vector_type(32)));
struct NativeArgs {
  uint64_t blk[32];
  uint32_t sl, n_tiles, seg_shift, seg_mask, seg_tiles;
  uint32_t n_parts;
};
// work item k -> tile: groups of 4 neighbouring tiles taken from
// 2^seg_shift segments in turn (the interpreter's order)
__device__ __forceinline__ uint32_t tile_of(uint32_t k, uint32_t shift, uint32_t mask, uint32_t seg_tiles) {
  const uint32_t g = k / 4u;
  return (g & mask) * seg_tiles + (g >> shift) * 4u + k % 4u;
}
)";

}  // namespace

std::string native_source(const std::vector<std::vector<uint32_t>> &parts, int K, int n_blocks) {
  const auto groups = slot_groups(K);
  std::string decl = "  v4u acc;", outs = "\"+{v[0:3]}\"(acc)", init_outs = "\"={v[0:3]}\"(acc)";
  for (size_t i = 0; i < groups.size(); ++i) {
    const int lo = groups[i].first, size = groups[i].second;
    decl += fmt(" v%du g%d;", size, (int)i);
    outs += fmt(", \"+{v[%d:%d]}\"(g%d)", lo, lo + size - 1, (int)i);
    init_outs += fmt(", \"={v[%d:%d]}\"(g%d)", lo, lo + size - 1, (int)i);
  }
  std::string init;
  for (int r = 0; r < 4 + 4 * K; ++r) init += fmt("v_mov_b32 v%d, 0\\n\\t", r);
  std::string ins;
  for (int c = 0; c < 8; ++c) ins += std::string(c ? ", " : "") + fmt("[o%d] \"v\"(o%d)", c, c);
  for (int b = 0; b < n_blocks; ++b) ins += fmt(", [b%d] \"s\"(b%d)", b, b);

  std::string s = kHead;
  s += "extern \"C\" __global__ void __launch_bounds__(256) ";
  s += kNativeKernel;
  s += "(NativeArgs a) {\n";
  s += "  const uint32_t lane = threadIdx.x & 63u;\n";
  s += "  const uint32_t wave = blockIdx.x * 4u + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));\n";
  s += "  const uint32_t n_waves = gridDim.x * 4u;\n";
  s += decl + "\n";
  s += "  // every slot starts at zero, and the program leaves it zero\n";
  s += "  asm volatile(\"" + init + "\" : " + init_outs + ");\n";
  for (int b = 0; b < n_blocks; ++b) s += fmt("  const uint64_t b%d = a.blk[%d];\n", b, b);
  s += "  const uint32_t voff = lane * 16u;\n";
  const bool split = parts.size() > 1;
  s += "  const uint32_t n_work = a.n_tiles * a.n_parts;\n";
  s += "  for (uint32_t k = wave; k < n_work; k += n_waves) {\n";
  if (split) {
    s += "    const uint32_t kt = k / a.n_parts, part = k - kt * a.n_parts;\n";
  } else {
    s += "    const uint32_t kt = k;\n";
  }
  s += "    const uint32_t toff = tile_of(kt, a.seg_shift, a.seg_mask, a.seg_tiles) * 1024u;\n";
  s += "    // lanes past the end of a ragged last tile sit the tile out\n";
  s += "    if (toff + voff < a.sl) {\n";
  s += "      // byte offset of this lane's 16 bytes of strip c in every block\n";
  for (int c = 0; c < 8; ++c) s += fmt("      const uint32_t o%d = toff + voff + %du * a.sl;\n", c, c);
  if (split) s += "      switch (part) {\n";
  for (size_t q = 0; q < parts.size(); ++q) {
    if (split) s += fmt("      case %d:\n", (int)q);
    s += "      asm volatile(\n";
    s += body(parts[q]);
    s += "        : " + outs + "\n";
    s += "        : " + ins + "\n";
    s += "        : \"memory\");\n";
    if (split) s += "      break;\n";
  }
  if (split) s += "      }\n";
  s += "    }\n  }\n}\n";
  return s;
}

ec_status native_compile(const std::string &src, std::vector<char> *code, std::string *log) {
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, src.c_str(), "ec_native.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return EC_ERR_NOMEM;
  // packed FP32 instructions off, as for every kernel of the library
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(p, (int)(sizeof opts / sizeof *opts), opts);
  size_t n = 0;
  if (log && hiprtcGetProgramLogSize(p, &n) == HIPRTC_SUCCESS && n > 1) {
    log->assign(n, '\0');
    hiprtcGetProgramLog(p, &(*log)[0]);
  }
  ec_status st = EC_OK;
  if (r != HIPRTC_SUCCESS || hiprtcGetCodeSize(p, &n) != HIPRTC_SUCCESS || n == 0) {
    st = EC_ERR_UNSUPPORTED;
  } else {
    code->resize(n);
    if (hiprtcGetCode(p, code->data()) != HIPRTC_SUCCESS) st = EC_ERR_UNSUPPORTED;
  }
  hiprtcDestroyProgram(&p);
  return st;
}

namespace {

struct Loaded {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int per_cu = 0;
};

// Never destroyed: programs may be launched or freed while the process exits.
std::mutex *const g_mu = new std::mutex;
std::map<std::pair<int, std::string>, Loaded> *const g_loaded = new std::map<std::pair<int, std::string>, Loaded>;

}  // namespace

ec_status native_function(int dev, const std::vector<char> &code, hipFunction_t *fn, int *per_cu) {
  std::lock_guard<std::mutex> g(*g_mu);
  const auto key = std::make_pair(dev, std::string(code.begin(), code.end()));
  auto it = g_loaded->find(key);
  if (it == g_loaded->end()) {
    Loaded l;
    if (hipModuleLoadData(&l.mod, code.data()) != hipSuccess) return EC_ERR_DEVICE;
    if (hipModuleGetFunction(&l.fn, l.mod, kNativeKernel) != hipSuccess ||
        hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&l.per_cu, l.fn, 256, 0) != hipSuccess ||
        l.per_cu < 1) {
      (void)hipModuleUnload(l.mod);
      return EC_ERR_DEVICE;
    }
    it = g_loaded->emplace(key, l).first;
  }
  *fn = it->second.fn;
  *per_cu = it->second.per_cu;
  return EC_OK;
}

int native_launch(hipFunction_t fn, const NativeArgs &a, int grid, hipStream_t stream) {
  NativeArgs arg = a;
  void *params[] = {&arg};
  return hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, 256, 1, 1, 0, stream, params, nullptr) == hipSuccess ? 0 : -1;
}

}  // namespace ec
