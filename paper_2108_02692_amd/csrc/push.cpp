// push.cpp -- push-form programs, their slot schedule and record encoding.
#include "push.hpp"

#include <algorithm>
#include <deque>
#include <functional>
#include <map>

#include "bytecode.hpp"

namespace ec {

namespace {

std::vector<int> cancel_pairs(const std::vector<int> &ops) {
  std::map<int, int> cnt;
  for (int o : ops) ++cnt[o];
  std::vector<int> out;
  for (int o : ops)
    if ((cnt[o] & 1) && std::find(out.begin(), out.end(), o) == out.end()) out.push_back(o);
  return out;
}

// Consumers of every value: strips first (index c), then accumulators
// (index n_const + a).
std::vector<std::vector<int>> consumers(const PushDag &d) {
  std::vector<std::vector<int>> cons(d.n_const + d.src.size());
  for (size_t a = 0; a < d.src.size(); ++a)
    for (int v : d.src[a]) cons[is_const(v) ? v - kConstBase : d.n_const + v].push_back((int)a);
  return cons;
}

}  // namespace

PushDag push_plain(const std::vector<Bits> &rows, int n_const) {
  PushDag d;
  d.n_const = n_const;
  d.n_rows = (int)rows.size();
  d.src.resize(rows.size());
  std::vector<char> used(n_const, 0);
  for (size_t r = 0; r < rows.size(); ++r)
    for (int c = 0; c < n_const; ++c)
      if (rows[r].test(c)) {
        d.src[r].push_back(kConstBase + c);
        used[c] = 1;
      }
  for (int c = 0; c < n_const; ++c)
    if (used[c]) d.order.push_back(c);
  return d;
}

PushDag push_blocked(const std::vector<Bits> &rows, int n_const, int width, bool rebuild, bool fused,
                     std::vector<Slp> *blocks) {
  const int R = (int)rows.size();
  PushDag d;
  d.n_const = n_const;
  d.n_rows = R;
  d.src.resize(R);
  for (int g0 = 0; g0 < n_const; g0 += width) {
    const int w = std::min(width, n_const - g0);
    std::vector<Bits> slice(R);
    for (int r = 0; r < R; ++r)
      for (int c = 0; c < w; ++c)
        if (rows[r].test(g0 + c)) slice[r].flip(c);
    Slp s = xor_repair(slice, w, rebuild);
    if (fused) s = fuse(s);
    if (blocks) blocks->push_back(s);
    // A statement that is only some row's own definition is inlined into that
    // row's accumulator; every other statement becomes a temporary.
    std::map<int, int> stmt_uses, out_uses;
    for (const Stmt &st : s.stmts)
      for (int o : st.ops)
        if (!is_const(o) && o != kZero) ++stmt_uses[o];
    for (int t : s.outputs)
      if (!is_const(t) && t != kZero) ++out_uses[t];
    std::map<int, int> acc_of;
    std::map<int, const Stmt *> inl;
    auto map_op = [&](int o) { return is_const(o) ? kConstBase + g0 + (o - kConstBase) : acc_of.at(o); };
    for (const Stmt &st : s.stmts) {
      if (stmt_uses[st.var] == 0 && out_uses[st.var] == 1) {
        inl[st.var] = &st;
        continue;
      }
      std::vector<int> ops;
      for (int o : st.ops)
        if (o != kZero) ops.push_back(map_op(o));
      acc_of[st.var] = (int)d.src.size();
      d.src.push_back(cancel_pairs(ops));
    }
    for (int r = 0; r < R; ++r) {
      const int t = s.outputs[r];
      if (t == kZero) continue;
      if (is_const(t)) {
        d.src[r].push_back(map_op(t));
      } else if (inl.count(t)) {
        for (int o : inl[t]->ops)
          if (o != kZero) d.src[r].push_back(map_op(o));
      } else {
        d.src[r].push_back(acc_of.at(t));
      }
    }
  }
  for (int r = 0; r < R; ++r) d.src[r] = cancel_pairs(d.src[r]);
  // A temporary that cancelled to nothing is the zero value: drop its uses.
  for (bool again = true; again;) {
    again = false;
    for (size_t a = R; a < d.src.size(); ++a) {
      if (!d.src[a].empty()) continue;
      for (auto &s2 : d.src) {
        auto it = std::find(s2.begin(), s2.end(), (int)a);
        if (it != s2.end()) { s2.erase(it); again = true; }
      }
    }
  }
  const std::vector<std::vector<int>> cons = consumers(d);
  for (int c = 0; c < n_const; ++c)
    if (!cons[c].empty()) d.order.push_back(c);
  return d;
}

namespace {

// Event-order simulation shared by the orderer and the scheduler's sizing:
// bring in strip c, then every temporary completed by it, recursively (FIFO).
struct DrySim {
  const PushDag &d;
  std::vector<std::vector<int>> cons;
  std::vector<int> pending;
  std::vector<char> open;
  int n_open = 0, peak = 0;
  explicit DrySim(const PushDag &dag) : d(dag), cons(consumers(dag)), pending(dag.src.size()), open(dag.src.size(), 0) {
    for (size_t a = 0; a < d.src.size(); ++a) pending[a] = (int)d.src[a].size();
  }
  // Returns (opened, completed) by value v (strip index or n_const + acc).
  std::pair<int, int> push(int v) {
    int opened = 0, completed = 0;
    std::deque<int> q{v};
    while (!q.empty()) {
      const int x = q.front();
      q.pop_front();
      if (x >= d.n_const) {  // a finished temporary leaves the register file
        open[x - d.n_const] = 0;
        --n_open;
      }
      for (int a : cons[x]) {
        if (a < d.n_rows) continue;
        if (!open[a]) { open[a] = 1; ++n_open; ++opened; }
        if (--pending[a] == 0) { q.push_back(d.n_const + a); ++completed; }
      }
      peak = std::max(peak, n_open);
    }
    return {opened, completed};
  }
};

}  // namespace

void push_unfold(PushDag &d, int record_cost) {
  const int R = d.n_rows;
  for (;;) {
    std::vector<int> uses(d.src.size(), 0);
    for (const auto &s : d.src)
      for (int v : s)
        if (!is_const(v)) ++uses[v];
    int best = -1;
    long best_gain = -1;
    for (size_t t = R; t < d.src.size(); ++t) {
      const long a = (long)d.src[t].size(), k = uses[t];
      if (a == 0 || k == 0) continue;
      const long gain = a + k + record_cost - a * k;
      if (gain > best_gain) { best_gain = gain; best = (int)t; }
    }
    if (best < 0) break;
    const std::vector<int> body = d.src[best];
    for (auto &s : d.src) {
      auto it = std::find(s.begin(), s.end(), best);
      if (it == s.end()) continue;
      std::vector<int> spliced(s.begin(), it);
      spliced.insert(spliced.end(), body.begin(), body.end());
      spliced.insert(spliced.end(), it + 1, s.end());
      s = cancel_pairs(spliced);
    }
    d.src[best].clear();
  }
  // drop the inlined temporaries and renumber the rest
  std::vector<int> newid(d.src.size(), -1);
  int next = R;
  for (int a = 0; a < R; ++a) newid[a] = a;
  for (size_t a = R; a < d.src.size(); ++a)
    if (!d.src[a].empty()) newid[a] = next++;
  std::vector<std::vector<int>> src(next);
  for (size_t a = 0; a < d.src.size(); ++a) {
    if (newid[a] < 0) continue;
    for (int v : d.src[a]) src[newid[a]].push_back(is_const(v) ? v : newid[v]);
  }
  d.src.swap(src);
}

void push_order(PushDag &d, int width) {
  DrySim sim(d);
  std::vector<int> order;
  size_t i = 0;
  while (i < d.order.size()) {
    const int blk = d.order[i] / width;
    std::vector<int> group;
    while (i < d.order.size() && d.order[i] / width == blk) group.push_back(d.order[i++]);
    while (!group.empty()) {
      size_t best = 0;
      int best_score = 1 << 30, best_done = -1;
      for (size_t k = 0; k < group.size(); ++k) {
        DrySim trial = sim;
        auto [op, done] = trial.push(group[k]);
        const int score = op - done;
        if (score < best_score || (score == best_score && done > best_done)) {
          best = k;
          best_score = score;
          best_done = done;
        }
      }
      sim.push(group[best]);
      order.push_back(group[best]);
      group.erase(group.begin() + best);
    }
  }
  d.order = order;
}

void push_order_greedy(PushDag &d, int width, int capacity) {
  const Slp g = greedy_schedule(push_as_slp(d), std::max(1, capacity));
  std::vector<char> used(d.n_const, 0), seen(d.n_const, 0);
  for (int c : d.order) used[c] = 1;
  std::vector<int> first;
  for (const Stmt &st : g.stmts)
    for (int o : st.ops)
      if (is_const(o) && used[o - kConstBase] && !seen[o - kConstBase]) {
        seen[o - kConstBase] = 1;
        first.push_back(o - kConstBase);
      }
  for (int c : d.order)  // (every strip in the order has a consumer, so none is left)
    if (!seen[c]) first.push_back(c);
  if (width > 0)
    std::stable_sort(first.begin(), first.end(), [width](int a, int b) { return a / width < b / width; });
  d.order = first;
}

std::vector<Bits> push_eval(const PushDag &d) {
  std::vector<Bits> val(d.src.size());
  std::vector<char> done(d.src.size(), 0);
  std::function<Bits(int)> get = [&](int a) -> Bits {
    if (done[a]) return val[a];
    Bits b;
    for (int v : d.src[a]) {
      if (is_const(v)) b.flip(v - kConstBase);
      else b = b ^ get(v);
    }
    done[a] = 1;
    return val[a] = b;
  };
  std::vector<Bits> rows;
  for (int r = 0; r < d.n_rows; ++r) rows.push_back(get(r));
  return rows;
}

Slp push_as_slp(const PushDag &d) {
  Slp s;
  s.n_const = d.n_const;
  DrySim sim(d);
  // temporaries in completion order
  std::vector<int> seq;
  {
    std::vector<int> pending(d.src.size());
    for (size_t a = 0; a < d.src.size(); ++a) pending[a] = (int)d.src[a].size();
    std::deque<int> q;
    for (int c : d.order) q.push_back(c);
    while (!q.empty()) {
      const int x = q.front();
      q.pop_front();
      for (int a : sim.cons[x])
        if (a >= d.n_rows && --pending[a] == 0) {
          seq.push_back(a);
          q.push_front(d.n_const + a);
        }
    }
  }
  for (int a : seq) s.stmts.push_back({a, d.src[a]});
  for (int r = 0; r < d.n_rows; ++r) {
    if (d.src[r].empty()) {
      s.outputs.push_back(kZero);
      continue;
    }
    s.stmts.push_back({r, d.src[r]});
    s.outputs.push_back(r);
  }
  return s;
}

// ------------------------------------------------------------------ scheduling
namespace {

struct Rec {
  uint32_t kind = bc::RUN;
  int pull = 0;
  std::vector<int> ops;
  int ld_slot = 0, blk = 0, j = 0;
  int wait_for = -1;  // VMEM sequence number of the pulled strip's load
  int ld_seq = -1;    // VMEM sequence number this record issues (LD or STORE)
};

enum SlotState { FREE_ZERO, FREE_DIRTY, LOADING, ACC };

struct Machine {
  int K;
  std::vector<int> state, last_pull, first_use;  // first_use: -1 none, 0 load, 1 needs zero
  std::vector<Rec> recs;
  int vm_seq = 0;
  explicit Machine(int k) : K(k), state(k, FREE_ZERO), last_pull(k, -1), first_use(k, -1) {}

  int pick(int want) const {
    for (int s = 0; s < K; ++s)
      if (state[s] == want) return s;
    return -1;
  }
  // A zero slot for an accumulator; a dirty one is cleared by XORing it into
  // itself in the record that last pulled it (that record's accumulator still
  // holds the slot's value).
  int take_zero() {
    int s = pick(FREE_ZERO);
    if (s < 0) {
      s = pick(FREE_DIRTY);
      if (s < 0 || last_pull[s] >= (int)recs.size()) return -1;
      recs[last_pull[s]].ops.push_back(s);
    }
    if (first_use[s] < 0) first_use[s] = 1;
    state[s] = ACC;
    return s;
  }
  int take_load() {
    int s = pick(FREE_DIRTY);
    if (s < 0) s = pick(FREE_ZERO);
    if (s < 0) return -1;
    if (first_use[s] < 0) first_use[s] = 0;
    state[s] = LOADING;
    return s;
  }
};

struct Pass {
  PushDag d;                 // rows of this pass are accumulators 0..R-1
  std::vector<int> row_out;  // global output row of each local row
};

// One pass: every output row accumulates in its own slot while all strips
// stream through.  Returns -1 if a slot is not available.
int run_pass(const Pass &ps, int n_in_blocks, int ring, int prefetch, Machine &m, int &peak_open, int &n_ops) {
  const PushDag &d = ps.d;
  const int R = d.n_rows;
  const std::vector<std::vector<int>> cons = consumers(d);
  std::vector<int> pending(d.src.size()), slot_of(d.src.size(), -1), strip_slot(d.n_const, -1),
      strip_seq(d.n_const, -1);
  for (size_t a = 0; a < d.src.size(); ++a) pending[a] = (int)d.src[a].size();
  for (int r = 0; r < R; ++r)
    if ((slot_of[r] = m.take_zero()) < 0) return -1;
  int n_open = 0;
  size_t next_load = 0, loaded = 0;  // strips whose load is issued / pulled
  auto issue = [&](Rec &rec) -> int {
    const int c = d.order[next_load];
    const int s = m.take_load();
    if (s < 0) return -1;
    rec.ld_slot = s;
    rec.blk = c / 8;
    rec.j = c % 8;
    rec.ld_seq = m.vm_seq++;
    strip_slot[c] = s;
    strip_seq[c] = rec.ld_seq;
    ++next_load;
    return 0;
  };
  // Prefetches run `prefetch` strips ahead of the register loads.
  size_t next_pf = 0;
  auto prefetch_upto = [&](size_t upto) {
    for (; next_pf < std::min(upto, d.order.size()); ++next_pf) {
      if (next_pf < next_load) continue;  // already loaded
      Rec pf;
      pf.kind = bc::PREFETCH;
      pf.blk = d.order[next_pf] / 8;
      pf.j = d.order[next_pf] % 8;
      pf.ld_seq = m.vm_seq++;
      m.recs.push_back(pf);
    }
  };
  // prologue: fill the ring
  while (next_load < d.order.size() && (int)(next_load - loaded) < ring) {
    Rec rec;
    rec.kind = bc::LOAD;
    if (issue(rec) < 0) return -1;
    m.recs.push_back(rec);
  }
  if (prefetch > 0) prefetch_upto(next_load + prefetch);
  // Run of the value held in the accumulator (pulled from slot `from`):
  // one XOR per consuming accumulator, opening temporaries as needed.
  // Temporaries it completes are appended to `done`.
  auto pushes = [&](Rec &rec, int value, int from, std::vector<int> &done) -> int {
    bool from_taken = false;
    for (int a : cons[value]) {
      if (slot_of[a] < 0) {  // a temporary opens
        if (from >= 0 && !from_taken && m.state[from] == FREE_DIRTY) {
          // the slot just pulled already holds this value: it becomes the
          // accumulator with no XOR at all
          slot_of[a] = from;
          m.state[from] = ACC;
          from_taken = true;
        } else {
          if ((slot_of[a] = m.take_zero()) < 0) return -1;
          rec.ops.push_back(slot_of[a]);
        }
        ++n_open;
        peak_open = std::max(peak_open, n_open);
      } else {
        rec.ops.push_back(slot_of[a]);
      }
      if (a >= R && --pending[a] == 0) done.push_back(a);
    }
    return 0;
  };
  // Finished temporaries, each pulled and pushed on in completion order.
  std::function<int(const std::vector<int> &)> finish = [&](const std::vector<int> &done) -> int {
    for (int a : done) {
      Rec v;
      v.kind = bc::VALUE;
      v.pull = slot_of[a];
      m.state[v.pull] = FREE_DIRTY;
      m.last_pull[v.pull] = (int)m.recs.size();
      --n_open;
      std::vector<int> more;
      if (pushes(v, d.n_const + a, v.pull, more) < 0) return -1;
      m.recs.push_back(v);
      if (finish(more) < 0) return -1;
    }
    return 0;
  };
  for (size_t i = 0; i < d.order.size(); ++i) {
    const int c = d.order[i];
    Rec rec;
    rec.kind = bc::INPUT;
    rec.pull = strip_slot[c];
    rec.wait_for = strip_seq[c];
    ++loaded;
    m.state[rec.pull] = FREE_DIRTY;
    m.last_pull[rec.pull] = (int)m.recs.size();
    std::vector<int> done;
    if (pushes(rec, c, rec.pull, done) < 0) return -1;
    // The refill is chosen after the run's accumulators (so the strip's own
    // slot can become one of them) and before any later record exists (so it
    // cannot take a slot that a later record still has to pull).  It cannot
    // take a slot of this run: those are accumulators, not free.
    if (next_load < d.order.size() && (int)(next_load - loaded) < ring) {
      rec.kind = bc::INPUT_LD;
      if (issue(rec) < 0) return -1;
    }
    n_ops += (int)rec.ops.size();
    m.recs.push_back(rec);
    if (prefetch > 0) prefetch_upto(next_load + prefetch);
    if (finish(done) < 0) return -1;
  }
  for (int r = 0; r < R; ++r) {
    Rec st;
    st.kind = bc::STORE;
    st.pull = slot_of[r];
    st.blk = n_in_blocks + ps.row_out[r] / 8;
    st.j = ps.row_out[r] % 8;
    st.ld_seq = m.vm_seq++;
    m.state[st.pull] = FREE_DIRTY;
    m.last_pull[st.pull] = (int)m.recs.size();
    m.recs.push_back(st);
  }
  return 0;
}

// Rows `rows` of `d` with the temporaries they need, renumbered.
Pass sub_dag(const PushDag &d, const std::vector<int> &rows) {
  Pass ps;
  ps.row_out = rows;
  std::vector<int> newid(d.src.size(), -1);
  std::vector<int> keep;
  for (size_t k = 0; k < rows.size(); ++k) newid[rows[k]] = (int)k;
  int next = (int)rows.size();
  std::function<void(int)> need = [&](int a) {
    for (int v : d.src[a])
      if (!is_const(v) && newid[v] < 0) {
        need(v);
        newid[v] = next++;
        keep.push_back(v);
      }
  };
  for (int r : rows) need(r);
  ps.d.n_const = d.n_const;
  ps.d.n_rows = (int)rows.size();
  ps.d.src.resize(next);
  auto remap = [&](int a) {
    std::vector<int> out;
    for (int v : d.src[a]) out.push_back(is_const(v) ? v : newid[v]);
    return out;
  };
  for (size_t k = 0; k < rows.size(); ++k) ps.d.src[k] = remap(rows[k]);
  for (int a : keep) ps.d.src[newid[a]] = remap(a);
  std::vector<char> used(d.n_const, 0);
  for (const auto &s : ps.d.src)
    for (int v : s)
      if (is_const(v)) used[v - kConstBase] = 1;
  for (int c : d.order)
    if (used[c]) ps.d.order.push_back(c);
  return ps;
}

int peak_open_temps(const PushDag &d) {
  DrySim sim(d);
  for (int c : d.order) sim.push(c);
  return sim.peak;
}

}  // namespace

int push_schedule(const PushDag &d, int n_in_blocks, const PushOpts &opts, PushCode &out) {
  const int K = opts.slots;
  const int R = opts.row_hi < 0 ? d.n_rows : std::min(opts.row_hi, d.n_rows);
  if (opts.row_lo < 0 || (opts.row_lo >= R && R > 0)) return -1;
  // Passes: as many rows per pass, in steps of 8 from row_lo (whole output
  // blocks when row_lo is a block boundary), as fit beside the pass's open
  // temporaries and a ring of at least two strips.
  std::vector<Pass> passes;
  for (int r0 = opts.row_lo; r0 < R;) {
    int take = 0;
    for (int nb = (R - r0 + 7) / 8; nb >= 1; --nb) {
      const int cnt = std::min(8 * nb, R - r0);
      std::vector<int> rows;
      for (int r = r0; r < r0 + cnt; ++r) rows.push_back(r);
      Pass ps = sub_dag(d, rows);
      if (cnt + peak_open_temps(ps.d) + 2 <= K) {
        passes.push_back(ps);
        take = cnt;
        break;
      }
    }
    if (take == 0) return -1;
    r0 += take;
  }
  Machine m(K);
  int peak_open = 0, n_ops = 0, ring_min = K;
  for (const Pass &ps : passes) {
    const int ring = std::min(opts.max_ring, K - ps.d.n_rows - peak_open_temps(ps.d));
    ring_min = std::min(ring_min, ring);
    if (run_pass(ps, n_in_blocks, ring, opts.prefetch, m, peak_open, n_ops) < 0) return -1;
  }
  // Leave every slot zero: the next tile may run another program (a batch
  // mixes them), and every program starts from all-zero slots.
  for (int s = 0; s < K; ++s)
    if (m.state[s] == FREE_DIRTY) m.recs[m.last_pull[s]].ops.push_back(s);

  // Encode; runs longer than one record continue in RUN records.
  std::vector<uint32_t> &w = out.words;
  w.clear();
  int vm_issued = 0, n_records = 0, n_loads = 0, n_stores = 0;
  out.n_prefetch = 0;
  for (const Rec &rec : m.recs) {
    uint32_t wait = 0;
    if (rec.kind == bc::INPUT || rec.kind == bc::INPUT_LD)
      wait = (uint32_t)std::min(bc::kMaxWait, vm_issued - rec.wait_for - 1);
    size_t k = 0;
    bool first = true;
    do {
      const size_t n = std::min<size_t>(bc::kMaxOps, rec.ops.size() - k);
      const uint32_t kind = first ? rec.kind : (uint32_t)bc::RUN;
      const bool has_ld = first && (kind == bc::INPUT_LD || kind == bc::LOAD);
      const bool has_blk = has_ld || (first && (kind == bc::STORE || kind == bc::PREFETCH));
      const uint32_t pull =
          (first && kind != bc::LOAD && kind != bc::RUN && kind != bc::PREFETCH) ? (uint32_t)rec.pull : 0u;
      w.push_back(bc::h0(kind, pull, (uint32_t)n));
      w.push_back(bc::h1(first ? wait : 0u, has_ld ? (uint32_t)rec.ld_slot : 0u, has_blk ? (uint32_t)rec.blk : 0u,
                         has_blk ? (uint32_t)rec.j : 0u));
      for (size_t q = 0; q < n; ++q) w.push_back(4u * (uint32_t)rec.ops[k + q]);
      k += n;
      first = false;
      ++n_records;
    } while (k < rec.ops.size());
    if (rec.kind == bc::INPUT_LD || rec.kind == bc::LOAD) { ++vm_issued; ++n_loads; }
    if (rec.kind == bc::STORE) { ++vm_issued; ++n_stores; }
    if (rec.kind == bc::PREFETCH) { ++vm_issued; ++out.n_prefetch; }
  }
  w.push_back(bc::h0(bc::HALT, 0, 0));
  w.push_back(0);
  w.insert(w.end(), bc::kWindow, 0u);
  int used = 0;
  for (int s = 0; s < K; ++s)
    if (m.first_use[s] >= 0) used = s + 1;
  out.slots_used = used;
  out.peak_open = peak_open;
  out.ring = ring_min;
  out.passes = (int)passes.size();
  out.n_loads = n_loads;
  out.n_stores = n_stores;
  out.n_records = n_records + 1;
  out.n_ops = 0;
  for (const Rec &rec : m.recs) out.n_ops += (int)rec.ops.size();
  return 0;
}

bool validate_code(const std::vector<uint32_t> &w, int slots, int n_in_blocks, int n_out_blocks) {
  size_t pc = 0;
  for (;;) {
    if (pc + bc::kWindow > w.size()) return false;
    const uint32_t a = w[pc], b = w[pc + 1];
    const uint32_t kind = bc::h0_kind(a);
    if (kind == bc::HALT) {
      if (a != bc::h0(bc::HALT, 0, 0) || b != 0) return false;
      for (size_t q = pc + 2; q < w.size(); ++q)
        if (w[q] != 0) return false;
      return w.size() - pc >= 2 + (size_t)bc::kWindow;
    }
    const uint32_t bytes = bc::h0_bytes(a);
    if (bytes < 8 || bytes > 8 + 4 * bc::kMaxOps || bytes % 4) return false;
    const uint32_t n = (bytes - 8) / 4;
    const uint32_t pull = bc::h0_pull(a);
    const bool pulls = kind == bc::INPUT || kind == bc::INPUT_LD || kind == bc::VALUE || kind == bc::STORE;
    const bool lds = kind == bc::INPUT_LD || kind == bc::LOAD;
    const bool waits = kind == bc::INPUT || kind == bc::INPUT_LD;
    if (a != bc::h0(kind, pulls ? pull : 0u, n)) return false;
    if (pulls && (int)pull >= slots) return false;
    const uint32_t wait = bc::h1_wait(b), ld = bc::h1_ld(b), blk = bc::h1_blk(b), j = bc::h1_j(b);
    if (b != bc::h1(wait, ld, blk, j)) return false;
    if (!waits && wait) return false;
    if (lds && ((int)ld >= slots || (int)blk >= n_in_blocks)) return false;
    if (!lds && ld) return false;
    if (kind == bc::STORE && ((int)blk < n_in_blocks || (int)blk >= n_in_blocks + n_out_blocks)) return false;
    if (kind == bc::PREFETCH && ((int)blk >= n_in_blocks || n)) return false;
    if (!lds && kind != bc::STORE && kind != bc::PREFETCH && (blk || j)) return false;
    if (pc + 2 + n > w.size()) return false;
    for (uint32_t q = 0; q < n; ++q) {
      const uint32_t o = w[pc + 2 + q];
      if (o % 4 || (int)(o / 4) >= slots) return false;
    }
    pc += 2 + n;
  }
}

bool simulate_code(const std::vector<uint32_t> &w, int slots, int n_in_blocks, int n_out_blocks,
                   const std::vector<Bits> &rows, int row_lo, int row_hi) {
  if (row_hi < 0) row_hi = (int)rows.size();
  if (!validate_code(w, slots, n_in_blocks, n_out_blocks)) return false;
  std::vector<Bits> slot(slots);
  std::vector<char> busy(slots, 0);     // a load into the slot is in flight
  for (int tile = 0; tile < 2; ++tile) {
    std::deque<int> vm;                 // outstanding VMEM operations (slot, or -1 for a store)
    std::vector<Bits> out(8 * n_out_blocks);
    std::vector<char> written(8 * n_out_blocks, 0);
    Bits acc;
    size_t pc = 0;
    for (;;) {
      const uint32_t a = w[pc], b = w[pc + 1];
      const uint32_t kind = bc::h0_kind(a);
      if (kind == bc::HALT) break;
      const uint32_t n = (bc::h0_bytes(a) - 8) / 4;
      if (kind == bc::INPUT || kind == bc::INPUT_LD) {
        const size_t keep = bc::h1_wait(b);
        while (vm.size() > keep) {
          if (vm.front() >= 0) busy[vm.front()] = 0;
          vm.pop_front();
        }
      }
      if (kind == bc::INPUT || kind == bc::INPUT_LD || kind == bc::VALUE || kind == bc::STORE) {
        const int s = (int)bc::h0_pull(a);
        if (busy[s]) return false;
        acc = slot[s];
      }
      if (kind == bc::INPUT_LD || kind == bc::LOAD) {
        const int s = (int)bc::h1_ld(b);
        if (busy[s]) return false;
        Bits v;
        v.flip(8 * (int)bc::h1_blk(b) + (int)bc::h1_j(b));
        slot[s] = v;  // lands later; reads before the wait are refused above
        busy[s] = 1;
        vm.push_back(s);
      }
      if (kind == bc::PREFETCH) vm.push_back(-1);
      if (kind == bc::STORE) {
        const int o = 8 * ((int)bc::h1_blk(b) - n_in_blocks) + (int)bc::h1_j(b);
        out[o] = acc;
        written[o] = 1;
        vm.push_back(-1);
      }
      for (uint32_t q = 0; q < n; ++q) {
        const int s = (int)(w[pc + 2 + q] / 4);
        if (busy[s]) return false;
        slot[s] = slot[s] ^ acc;
      }
      pc += 2 + n;
    }
    for (int r = 0; r < (int)written.size(); ++r) {
      const bool want = r >= row_lo && r < row_hi && r < (int)rows.size();
      if (want != (bool)written[r] || (want && !(out[r] == rows[r]))) return false;
    }
    for (int s = 0; s < slots; ++s)
      if (busy[s] || !(slot[s] == Bits())) return false;  // loads consumed, slots left zero
  }
  return true;
}

}  // namespace ec
