// sched.cpp -- GPU form of the pebble game (Secs. 6.3-6.6).
//
// The paper's pebbles are cache blocks under an LRU rule; here they are K
// VGPR slots (16 bytes per lane each) whose evictions the compiler chooses,
// i.e. the red-blue game with chosen eviction the paper relates its game to.
// Each statement streams its operands into an accumulator, so a value needs
// a slot only from its load or computation to its last read:
//  * a temporary keeps its slot until its last read (never evicted);
//  * an input strip is loaded into a free slot, or, when none is free, into
//    the slot of the resident input whose next read is farthest away
//    (Belady); evicted inputs are loaded again later (an L2 hit, not HBM);
//  * a load is issued as early as its slot allows, up to `hoist` ops ahead of
//    its first read, so its latency overlaps the XORs in between (the
//    software prefetching the paper leaves to future work);
//  * the vector-memory counter is modelled exactly, and a WAIT is placed
//    before the first read of each loaded slot.
#include "sched.hpp"

#include <algorithm>
#include <climits>
#include <map>
#include <unordered_map>

#include "bytecode.hpp"

namespace ec {
namespace {

struct XStmt {
  std::vector<int> ops;     // terms
  int var;                  // -1 for output copies
  bool put;                 // value read by later statements
  std::vector<int> stores;  // output strips
};

struct Pos {
  int stmt;     // index into xs
  int operand;  // operand index, or -1 for the END group
};

enum Kind { FREE_NEVER, IN, TMP };

struct Slot {
  Kind kind = FREE_NEVER;
  int id = -1;
  bool live = false;   // holds a value that is read later
  int last_read = -1;  // last position the current value was read or written
};

struct Load {
  int slot, strip, issue_min, use;
};

}  // namespace

int schedule(const Slp &p, int n_in_strips, int n_out_strips, const SchedOpts &opts, SchedResult &out) {
  const int K = opts.slots;
  // ---- statements to execute
  std::unordered_map<int, int> last_use_stmt;
  for (size_t i = 0; i < p.stmts.size(); ++i)
    for (int o : p.stmts[i].ops)
      if (!is_const(o) && o != kZero) last_use_stmt[o] = (int)i;
  std::map<int, std::vector<int>> outs_of;  // term -> output strips
  for (int o = 0; o < (int)p.outputs.size(); ++o) outs_of[p.outputs[o]].push_back(o);

  std::vector<XStmt> xs;
  for (const Stmt &s : p.stmts) {
    XStmt x{s.ops, s.var, last_use_stmt.count(s.var) > 0, {}};
    auto it = outs_of.find(s.var);
    if (it != outs_of.end()) x.stores = it->second;
    if (!x.put && x.stores.empty()) continue;  // dead
    xs.push_back(x);
  }
  for (const auto &kv : outs_of) {
    const int t = kv.first;
    if (t == kZero) xs.push_back({{}, -1, false, kv.second});
    else if (is_const(t)) xs.push_back({{t}, -1, false, kv.second});
  }

  // ---- positions and read lists
  std::vector<Pos> pos;
  std::unordered_map<int, std::vector<int>> in_reads;  // strip -> positions
  std::unordered_map<int, int> tmp_last;               // var -> last read position
  for (int i = 0; i < (int)xs.size(); ++i) {
    for (int k = 0; k < (int)xs[i].ops.size(); ++k) {
      const int t = xs[i].ops[k];
      const int q = (int)pos.size();
      if (is_const(t)) in_reads[t - kConstBase].push_back(q);
      else tmp_last[t] = q;
      pos.push_back({i, k});
    }
    pos.push_back({i, -1});
  }
  auto next_read = [&](int strip, int q) {
    const std::vector<int> &r = in_reads[strip];
    auto it = std::upper_bound(r.begin(), r.end(), q);
    return it == r.end() ? INT_MAX : *it;
  };

  // ---- allocation
  std::vector<Slot> slot(K);
  std::unordered_map<int, int> in_slot, tmp_slot;
  std::vector<Load> loads;
  std::vector<int> put_slot(xs.size(), -1);
  std::vector<int> read_slot(pos.size(), -1);
  int peak = 0;

  auto pick_free = [&](bool earliest) {
    int best = -1;
    for (int s = 0; s < K; ++s) {
      if (slot[s].live) continue;
      if (best < 0) { best = s; continue; }
      const bool better = earliest ? slot[s].last_read < slot[best].last_read
                                   : slot[s].last_read > slot[best].last_read;
      if (better) best = s;
    }
    return best;
  };
  auto evict_belady = [&](int q) {
    int best = -1, far = -1;
    for (int s = 0; s < K; ++s) {
      if (!slot[s].live || slot[s].kind != IN) continue;
      const int nr = next_read(slot[s].id, q);
      if (nr > far) { far = nr; best = s; }
    }
    if (best >= 0) in_slot.erase(slot[best].id);
    return best;
  };
  auto live_count = [&]() {
    int n = 0;
    for (const Slot &s : slot) n += s.live;
    return n;
  };

  for (int q = 0; q < (int)pos.size(); ++q) {
    const XStmt &x = xs[pos[q].stmt];
    if (pos[q].operand >= 0) {
      const int t = x.ops[pos[q].operand];
      int s;
      if (!is_const(t)) {
        s = tmp_slot.at(t);
        if (tmp_last[t] == q) slot[s].live = false;
      } else {
        const int c = t - kConstBase;
        auto it = in_slot.find(c);
        if (it != in_slot.end()) {
          s = it->second;
        } else {
          s = pick_free(true);
          if (s < 0) s = evict_belady(q);
          if (s < 0) return -1;
          loads.push_back({s, c, slot[s].last_read + 1, q});
          slot[s].kind = IN;
          slot[s].id = c;
          slot[s].live = true;
          in_slot[c] = s;
        }
        if (next_read(c, q) == INT_MAX) {
          slot[s].live = false;
          in_slot.erase(c);
        }
      }
      slot[s].last_read = q;
      read_slot[q] = s;
      peak = std::max(peak, live_count() + (slot[s].live ? 0 : 1));
    } else if (x.put) {
      int s = pick_free(false);
      if (s < 0) s = evict_belady(q);
      if (s < 0) return -1;
      slot[s].kind = TMP;
      slot[s].id = x.var;
      slot[s].live = true;
      slot[s].last_read = q;
      tmp_slot[x.var] = s;
      put_slot[pos[q].stmt] = s;
      peak = std::max(peak, live_count());
    }
  }

  // ---- emission with hoisted loads and exact vmcnt waits
  const int H = std::max(0, opts.hoist);
  std::vector<std::vector<int>> loads_at(pos.size());
  for (int i = 0; i < (int)loads.size(); ++i) {
    const int at = std::max(loads[i].issue_min, loads[i].use - H);
    loads_at[std::min(at, loads[i].use)].push_back(i);
  }
  std::vector<bc::Micro> ops;
  auto micro = [](bc::Kind k, int slot, int strip, int count) {
    return bc::Micro{k, (int16_t)slot, (int16_t)strip, (int16_t)count};
  };
  std::vector<long> pending(K, -1);  // vm op sequence of the last load into a slot
  long issued = 0, completed = -1;
  const long maxq = std::min(opts.max_inflight, bc::kMaxVmcnt);
  auto throttle = [&]() {
    if (issued - 1 - completed >= maxq) {
      ops.push_back(micro(bc::WAIT, 0, 0, (int)maxq - 1));
      completed = issued - maxq;
    }
  };
  int n_loads = 0, n_stores = 0;
  for (int q = 0; q < (int)pos.size(); ++q) {
    for (int li : loads_at[q]) {
      throttle();
      ops.push_back(micro(bc::LD, loads[li].slot, loads[li].strip, 0));
      pending[loads[li].slot] = issued++;
      ++n_loads;
    }
    const XStmt &x = xs[pos[q].stmt];
    if (pos[q].operand >= 0) {
      const int s = read_slot[q];
      if (pending[s] > completed) {
        ops.push_back(micro(bc::WAIT, 0, 0, (int)(issued - 1 - pending[s])));
        completed = pending[s];
      }
      ops.push_back(micro(bc::PULL, s, 0, 0));
    } else {
      const int ps = put_slot[pos[q].stmt];
      if (ps >= 0) {
        pending[ps] = -1;
        ops.push_back(micro(bc::PUT, ps, 0, 0));
      }
      for (int o : x.stores) {
        throttle();
        ops.push_back(micro(bc::STORE, 0, o, 0));
        ++issued;
        ++n_stores;
      }
      ops.push_back(micro(bc::CLEAR, 0, 0, 0));
    }
  }
  ops.push_back(micro(bc::HALT, 0, 0, 0));
  out.words = bc::pack(ops);

  int used = 0;
  for (int s = 0; s < K; ++s)
    if (slot[s].kind != FREE_NEVER) used = s + 1;
  out.slots_used = used;
  out.peak_live = peak;
  out.n_loads = n_loads;
  out.n_stores = n_stores;
  if (!validate_bytecode(out.words, K, n_in_strips, n_out_strips)) return -2;
  return 0;
}

namespace bc {

std::vector<uint32_t> pack(const std::vector<Micro> &ops) {
  std::vector<uint32_t> w;
  size_t i = 0;
  const size_t N = ops.size();
  while (i < N) {
    uint32_t h0 = 0, h1 = 0;
    std::vector<uint32_t> pulls, pushes;
    int stage = 0;  // canonical order: LD WAIT PULL PUT STORE PUSH CLEAR HALT
    bool set_mode = false;
    for (; i < N; ++i) {
      const Micro &m = ops[i];
      const bool room = pulls.size() + pushes.size() < (size_t)kMaxOperands;
      if (m.kind == LD && stage < 1) {
        h0 |= H0_LD | ((uint32_t)m.slot << 9) | ((uint32_t)m.strip << 15);
        stage = 1;
      } else if (m.kind == WAIT && stage < 2) {
        h0 |= H0_WAIT;
        h1 |= (uint32_t)m.count;
        stage = 2;
      } else if (m.kind == PULL && stage <= 2 && room) {
        pulls.push_back((uint32_t)(4 * m.slot));
        stage = 2;
      } else if (m.kind == PUT && stage < 4) {
        h1 |= H1_PUT | ((uint32_t)m.slot << 7);
        stage = 4;
      } else if (m.kind == STORE && stage < 5) {
        h1 |= H1_STORE | ((uint32_t)m.strip << 14);
        stage = 5;
      } else if ((m.kind == PUSH || m.kind == PUSHSET) && stage <= 5 && room &&
                 (pushes.empty() || set_mode == (m.kind == PUSHSET))) {
        set_mode = m.kind == PUSHSET;
        pushes.push_back((uint32_t)(4 * m.slot));
        stage = 5;
      } else if (m.kind == CLEAR && stage < 7) {
        h1 |= H1_CLEAR;
        stage = 7;
      } else if (m.kind == HALT && stage < 8) {
        h1 |= H1_HALT;
        stage = 8;
      } else {
        break;
      }
    }
    h0 |= (uint32_t)pulls.size() | ((uint32_t)pushes.size() << 4) | (set_mode ? H0_SET : 0u);
    const size_t base = w.size();
    w.resize(base + kBlockWords, 0u);
    w[base] = h0;
    w[base + 1] = h1;
    for (size_t k = 0; k < pulls.size(); ++k) w[base + 2 + k] = pulls[k];
    for (size_t k = 0; k < pushes.size(); ++k) w[base + kBlockWords - pushes.size() + k] = pushes[k];
  }
  w.resize(w.size() + kBlockWords, 0u);  // read-ahead block after HALT
  return w;
}

}  // namespace bc

bool validate_bytecode(const std::vector<uint32_t> &w, int slots, int n_in_strips, int n_out_strips) {
  // Walk the blocks exactly as the device does; the device trusts every field.
  if (w.size() % bc::kBlockWords != 0) return false;
  auto slot_word_ok = [&](uint32_t o) { return (o & ~0xFCu) == 0 && (int)(o >> 2) < slots; };
  for (size_t pc = 0;; pc += bc::kBlockWords) {
    if (pc + 2 * bc::kBlockWords > w.size()) return false;  // the device reads one block ahead
    const uint32_t h0 = w[pc], h1 = w[pc + 1];
    const uint32_t np = bc::h0_np(h0), nq = bc::h0_nq(h0);
    if (np + nq > (uint32_t)bc::kMaxOperands) return false;
    if (h0 >> 28) return false;
    if (h0 & bc::H0_LD) {
      if ((int)bc::h0_ld_slot(h0) >= slots || (int)bc::h0_ld_strip(h0) >= n_in_strips) return false;
    } else if (h0 & 0x03FFFE00u) {
      return false;
    }
    if (!(h0 & bc::H0_WAIT) && bc::h1_wait(h1)) return false;
    if (h1 >> 27) return false;
    if (h1 & bc::H1_PUT) {
      if ((int)bc::h1_put_slot(h1) >= slots) return false;
    } else if (h1 & 0x1F80u) {
      return false;
    }
    if (h1 & bc::H1_STORE) {
      if ((int)bc::h1_store_strip(h1) >= n_out_strips) return false;
    } else if (h1 & 0x01FFC000u) {
      return false;
    }
    for (uint32_t k = 0; k < (uint32_t)bc::kMaxOperands; ++k) {
      const uint32_t o = w[pc + 2 + k];
      const bool used = k < np || k >= (uint32_t)bc::kMaxOperands - nq;
      if (used ? !slot_word_ok(o) : o != 0) return false;
    }
    if (h1 & bc::H1_HALT) return pc + 2 * bc::kBlockWords == w.size();
  }
}

// ---------------------------------------------------------------- broadcast form
int schedule_broadcast(const std::vector<Bits> &rows, int n_in_strips, const SchedOpts &opts, SchedResult &out) {
  const int R = (int)rows.size();
  const int K = opts.slots;
  const int Q = K - R;  // ring of prefetch slots for input strips
  if (Q < 2) return -1;
  std::vector<int> inputs;
  std::vector<std::vector<int>> targets;
  for (int c = 0; c < n_in_strips; ++c) {
    std::vector<int> t;
    for (int j = 0; j < R; ++j)
      if (rows[j].test(c)) t.push_back(j);
    if (!t.empty()) { inputs.push_back(c); targets.push_back(t); }
  }
  const int U = (int)inputs.size();
  std::vector<bc::Micro> ops;
  auto m = [](bc::Kind k, int slot, int strip, int count) {
    return bc::Micro{k, (int16_t)slot, (int16_t)strip, (int16_t)count};
  };
  long issued = 0;
  std::vector<long> seq(U, -1);
  auto ring = [&](int i) { return R + (i % Q); };
  // Prefetch the first Q inputs, interleaved with zeroing the accumulators
  // (acc is 0 at tile start, so PUSHSET writes zeros).
  int z = 0, pre = 0;
  while (z < R || pre < std::min(Q, U)) {
    if (pre < std::min(Q, U)) {
      ops.push_back(m(bc::LD, ring(pre), inputs[pre], 0));
      seq[pre++] = issued++;
    }
    for (int k = 0; k < bc::kMaxOperands && z < R; ++k) ops.push_back(m(bc::PUSHSET, z++, 0, 0));
  }
  for (int i = 0; i < U; ++i) {
    if (i >= 1 && i - 1 + Q < U) {  // refill the slot input i-1 just left
      ops.push_back(m(bc::LD, ring(i - 1), inputs[i - 1 + Q], 0));
      seq[i - 1 + Q] = issued++;
    }
    ops.push_back(m(bc::WAIT, 0, 0, (int)(issued - 1 - seq[i])));
    ops.push_back(m(bc::PULL, ring(i), 0, 0));
    for (int j : targets[i]) ops.push_back(m(bc::PUSH, j, 0, 0));
    ops.push_back(m(bc::CLEAR, 0, 0, 0));
  }
  for (int j = 0; j < R; ++j) {
    ops.push_back(m(bc::PULL, j, 0, 0));
    ops.push_back(m(bc::STORE, 0, j, 0));
    ops.push_back(m(bc::CLEAR, 0, 0, 0));
  }
  ops.push_back(m(bc::HALT, 0, 0, 0));
  out.words = bc::pack(ops);
  out.slots_used = R + std::min(Q, U);
  out.peak_live = out.slots_used;
  out.n_loads = U;
  out.n_stores = R;
  if (!validate_bytecode(out.words, K, n_in_strips, R)) return -2;
  return 0;
}

}  // namespace ec
