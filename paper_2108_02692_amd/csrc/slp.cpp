// slp.cpp -- bitmatrix expansion, plain SLP, (Xor)RePair, XOR fusion and DFS
// scheduling (Secs. 1, 2, 4, 5 and 6 of the paper).
//
// Readings of points the paper leaves open:
//  * term order: temporaries by creation, all before constants; constants by
//    strip index 8*block + strip (Sec. 4.3);
//  * a pair's frequency is the number of original definitions holding both
//    terms; ties go to the lexicographically smallest pair;
//  * Rebuild (Sec. 4.4) scans every temporary, takes the one leaving the
//    smallest remainder (ties: earliest), and its result replaces the
//    definition only when strictly shorter;
//  * fusion (Sec. 5.2) never unfolds a returned variable, splices the
//    unfolded operands at the variable's position, cancels repeated operands
//    and always unfolds the earliest eligible statement first.
#include "slp.hpp"

#include <algorithm>
#include <map>
#include <set>
#include <unordered_map>

namespace ec {

std::vector<Bits> bitmatrix_rows(int rows, int cols, const Mat &m) {
  std::vector<Bits> out((size_t)rows * 8);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) {
      const uint8_t e = m[(size_t)i * cols + j];
      for (int c = 0; c < 8; ++c) {
        const uint8_t col = gf::mul(e, (uint8_t)(1u << c));
        for (int r = 0; r < 8; ++r)
          if ((col >> r) & 1u) out[(size_t)8 * i + r].flip(8 * j + c);
      }
    }
  return out;
}

Slp plain_slp(const std::vector<Bits> &rows, int n_const) {
  Slp p;
  p.n_const = n_const;
  for (size_t r = 0; r < rows.size(); ++r) {
    std::vector<int> ops;
    for (int c = 0; c < n_const; ++c)
      if (rows[r].test(c)) ops.push_back(kConstBase + c);
    if (ops.empty()) {
      p.outputs.push_back(kZero);
      continue;
    }
    p.stmts.push_back({(int)r, ops});
    p.outputs.push_back((int)r);
  }
  return p;
}

// ---------------------------------------------------------------- (Xor)RePair
Slp xor_repair(const std::vector<Bits> &rows, int n_const, bool rebuild) {
  const int R = (int)rows.size();
  int total = 0;
  for (const Bits &b : rows) total += b.count();
  // Dense term ids: temporaries [0, tcap), constant c -> tcap + c.  Each
  // pairing shrinks the total definition size, so at most `total` temps.
  const int tcap = total + 1;
  const int D = tcap + n_const;
  std::vector<uint16_t> cnt((size_t)D * D, 0);

  std::vector<std::vector<int>> defs(R);
  std::vector<char> active(R, 1);
  std::vector<int> alias(R, kZero);
  for (int i = 0; i < R; ++i)
    for (int c = 0; c < n_const; ++c)
      if (rows[i].test(c)) defs[i].push_back(tcap + c);

  std::vector<std::pair<int, int>> temps;
  std::vector<Bits> tval;
  auto val = [&](int d) -> Bits {
    if (d < tcap) return tval[d];
    Bits b;
    b.flip(d - tcap);
    return b;
  };
  auto settle = [&]() {
    for (int i = 0; i < R; ++i)
      if (active[i] && defs[i].size() <= 1) {
        alias[i] = defs[i].empty() ? -1 : defs[i][0];
        active[i] = 0;
      }
  };
  auto do_rebuild = [&](int i) {
    Bits rem = rows[i];
    std::vector<int> chosen;
    for (;;) {
      int best = -1, best_sz = rem.count();
      for (int k = 0; k < (int)tval.size(); ++k) {
        const int sz = (rem ^ tval[k]).count();
        if (sz < best_sz) { best = k; best_sz = sz; }
      }
      if (best < 0) break;
      rem = rem ^ tval[best];
      chosen.push_back(best);
    }
    std::vector<int> nd(chosen.begin(), chosen.end());
    for (int c = 0; c < n_const; ++c)
      if (rem.test(c)) nd.push_back(tcap + c);
    std::sort(nd.begin(), nd.end());
    return nd;
  };

  settle();
  for (;;) {
    bool any = false;
    for (int i = 0; i < R; ++i) any |= (bool)active[i];
    if (!any) break;
    // Most frequent pair, ties to the smallest (x, y).
    int best_f = 0;
    size_t best_key = (size_t)-1;
    for (int i = 0; i < R; ++i) {
      if (!active[i]) continue;
      const std::vector<int> &d = defs[i];
      for (size_t a = 0; a < d.size(); ++a)
        for (size_t b = a + 1; b < d.size(); ++b) {
          const size_t k = (size_t)d[a] * D + d[b];
          const int c = ++cnt[k];
          if (c > best_f || (c == best_f && k < best_key)) { best_f = c; best_key = k; }
        }
    }
    for (int i = 0; i < R; ++i) {
      if (!active[i]) continue;
      const std::vector<int> &d = defs[i];
      for (size_t a = 0; a < d.size(); ++a)
        for (size_t b = a + 1; b < d.size(); ++b) cnt[(size_t)d[a] * D + d[b]] = 0;
    }
    const int x = (int)(best_key / D), y = (int)(best_key % D);
    const int t = (int)temps.size();
    temps.push_back({x, y});
    tval.push_back(val(x) ^ val(y));
    for (int i = 0; i < R; ++i) {
      if (!active[i]) continue;
      std::vector<int> &d = defs[i];
      auto ix = std::lower_bound(d.begin(), d.end(), x);
      auto iy = std::lower_bound(d.begin(), d.end(), y);
      if (ix == d.end() || *ix != x || iy == d.end() || *iy != y) continue;
      d.erase(iy);
      d.erase(std::lower_bound(d.begin(), d.end(), x));
      d.insert(std::lower_bound(d.begin(), d.end(), t), t);
    }
    if (rebuild)
      for (int i = 0; i < R; ++i) {
        if (!active[i]) continue;
        std::vector<int> nd = do_rebuild(i);
        if (nd.size() < defs[i].size()) defs[i] = nd;
      }
    settle();
  }

  auto term = [&](int d) { return d < 0 ? kZero : (d < tcap ? d : kConstBase + (d - tcap)); };
  Slp out;
  out.n_const = n_const;
  for (int k = 0; k < (int)temps.size(); ++k)
    out.stmts.push_back({k, {term(temps[k].first), term(temps[k].second)}});
  for (int i = 0; i < R; ++i) out.outputs.push_back(term(alias[i]));
  return out;
}

// ---------------------------------------------------------------- fusion
static std::vector<int> cancel_ops(const std::vector<int> &ops) {
  std::map<int, int> cnt;
  for (int o : ops) ++cnt[o];
  std::vector<int> out;
  for (int o : ops)
    if ((cnt[o] & 1) && std::find(out.begin(), out.end(), o) == out.end()) out.push_back(o);
  return out;
}

Slp fuse(const Slp &in) {
  Slp p = in;
  std::set<int> outset(in.outputs.begin(), in.outputs.end());
  for (;;) {
    std::unordered_map<int, int> uses;
    for (const Stmt &s : p.stmts)
      for (int o : s.ops)
        if (!is_const(o) && o != kZero) ++uses[o];
    bool removed = false;
    std::vector<Stmt> kept;
    for (const Stmt &s : p.stmts) {
      if (uses[s.var] == 0 && !outset.count(s.var)) { removed = true; continue; }
      kept.push_back(s);
    }
    if (removed) { p.stmts.swap(kept); continue; }
    int target = -1;
    for (size_t i = 0; i < p.stmts.size(); ++i)
      if (!outset.count(p.stmts[i].var) && uses[p.stmts[i].var] == 1) { target = (int)i; break; }
    if (target < 0) break;
    const Stmt v = p.stmts[target];
    for (Stmt &w : p.stmts) {
      auto it = std::find(w.ops.begin(), w.ops.end(), v.var);
      if (it == w.ops.end()) continue;
      std::vector<int> spliced(w.ops.begin(), it);
      spliced.insert(spliced.end(), v.ops.begin(), v.ops.end());
      spliced.insert(spliced.end(), it + 1, w.ops.end());
      w.ops = cancel_ops(spliced);
      break;
    }
    p.stmts.erase(p.stmts.begin() + target);
  }
  return p;
}

// ---------------------------------------------------------------- DFS
Slp dfs_schedule(const Slp &in) {
  std::map<int, const Stmt *> by_var;
  for (const Stmt &s : in.stmts) by_var[s.var] = &s;
  std::set<int> used;
  for (const Stmt &s : in.stmts)
    for (int o : s.ops)
      if (by_var.count(o)) used.insert(o);
  // roots: the returned variables in the order they are returned, then the
  // other statements no statement uses, by variable (map order)
  std::vector<int> roots;
  std::set<int> is_root;
  for (int o : in.outputs)
    if (by_var.count(o) && is_root.insert(o).second) roots.push_back(o);
  for (const auto &kv : by_var)
    if (!used.count(kv.first) && is_root.insert(kv.first).second) roots.push_back(kv.first);
  std::set<int> seen;
  Slp out;
  out.n_const = in.n_const;
  out.outputs = in.outputs;
  for (int r : roots) {
    std::vector<std::pair<int, bool>> stack{{r, false}};
    while (!stack.empty()) {
      auto [node, done] = stack.back();
      stack.pop_back();
      if (done) { out.stmts.push_back(*by_var[node]); continue; }
      if (seen.count(node)) continue;
      seen.insert(node);
      stack.push_back({node, true});
      std::vector<int> kids;
      for (int o : by_var[node]->ops)
        if (by_var.count(o)) kids.push_back(o);
      std::sort(kids.begin(), kids.end());
      for (auto it = kids.rbegin(); it != kids.rend(); ++it)
        if (!seen.count(*it)) stack.push_back({*it, false});
    }
  }
  return out;
}

// ---------------------------------------------------------------- greedy
Slp greedy_schedule(const Slp &in, int capacity) {
  // Each step computes one ready node (all variable children computed):
  // the one whose children are most often already cached, as a fraction of
  // its distinct children, ties to the earliest variable.  Its children are
  // touched cached ones first, then the rest, each group in term order, and
  // its value goes on a dead pebble (holding a variable neither returned nor
  // used again), a cached one first, ties to the earliest held variable;
  // else on a fresh pebble.
  const int ns = (int)in.stmts.size();
  auto before = [](int a, int b) {
    const bool ca = is_const(a), cb = is_const(b);
    return ca != cb ? cb : a < b;  // temporaries before constants, each by number
  };
  std::vector<std::vector<int>> kids(ns);
  std::unordered_map<int, int> uses;
  for (int i = 0; i < ns; ++i)
    for (int o : in.stmts[i].ops) {
      if (o == kZero || std::find(kids[i].begin(), kids[i].end(), o) != kids[i].end()) continue;
      kids[i].push_back(o);
      if (!is_const(o)) ++uses[o];
    }
  std::set<int> goals;
  for (int o : in.outputs)
    if (o != kZero && !is_const(o)) goals.insert(o);
  std::vector<int> todo(ns);
  for (int i = 0; i < ns; ++i) todo[i] = i;
  std::sort(todo.begin(), todo.end(), [&](int a, int b) { return in.stmts[a].var < in.stmts[b].var; });

  // LRU cache of constants (as themselves) and pebbles (q as -(q + 2)),
  // each with the time of its last touch
  std::unordered_map<int, long> stamp;
  long clock = 0;
  auto touch = [&](int e) {
    if (!stamp.count(e) && (int)stamp.size() >= capacity) {
      auto lru = stamp.begin();
      for (auto it = stamp.begin(); it != stamp.end(); ++it)
        if (it->second < lru->second) lru = it;
      stamp.erase(lru);
    }
    stamp[e] = ++clock;
  };
  std::unordered_map<int, int> peb;  // variable -> pebble
  std::vector<int> held;             // pebble -> variable on it
  auto entry = [&](int t) { return is_const(t) ? t : -(peb.at(t) + 2); };

  Slp out;
  out.n_const = in.n_const;
  while (!todo.empty()) {
    int best = -1;
    long bh = 0, bc = 1;
    for (int k = 0; k < (int)todo.size(); ++k) {
      const std::vector<int> &c = kids[todo[k]];
      bool ready = true;
      long h = 0;
      for (int o : c) {
        if (!is_const(o) && !peb.count(o)) { ready = false; break; }
        h += stamp.count(entry(o));
      }
      if (!ready) continue;
      const long n = std::max<long>((long)c.size(), 1);
      if (best < 0 || h * bc > bh * n) { best = k; bh = h; bc = n; }
    }
    const int i = todo[best];
    todo.erase(todo.begin() + best);
    std::vector<int> hit, miss;
    for (int o : kids[i]) (stamp.count(entry(o)) ? hit : miss).push_back(o);
    std::sort(hit.begin(), hit.end(), before);
    std::sort(miss.begin(), miss.end(), before);
    hit.insert(hit.end(), miss.begin(), miss.end());
    Stmt s;
    for (int o : hit) {
      touch(entry(o));
      s.ops.push_back(is_const(o) ? o : peb.at(o));
    }
    for (int o : kids[i])
      if (!is_const(o)) --uses[o];
    int pick = -1;
    bool pick_cached = false;
    for (int q = 0; q < (int)held.size(); ++q) {
      const int u = held[q];
      if (goals.count(u) || uses[u] != 0) continue;
      const bool c = stamp.count(-(q + 2)) != 0;
      if (pick < 0 || (c && !pick_cached) || (c == pick_cached && before(u, held[pick]))) {
        pick = q;
        pick_cached = c;
      }
    }
    if (pick < 0) {
      pick = (int)held.size();
      held.push_back(0);
    }
    touch(-(pick + 2));
    held[pick] = in.stmts[i].var;
    peb[in.stmts[i].var] = pick;
    s.var = pick;
    out.stmts.push_back(std::move(s));
  }
  for (int o : in.outputs) out.outputs.push_back(o == kZero || is_const(o) ? o : peb.at(o));
  return out;
}

// ---------------------------------------------------------------- measures
std::vector<Bits> evaluate(const Slp &p) {
  std::unordered_map<int, Bits> env;
  auto val = [&](int t) {
    Bits b;
    if (t == kZero) return b;
    if (is_const(t)) { b.flip(t - kConstBase); return b; }
    return env.at(t);
  };
  for (const Stmt &s : p.stmts) {
    Bits x;
    for (int o : s.ops) x = x ^ val(o);
    env[s.var] = x;
  }
  std::vector<Bits> out;
  for (int t : p.outputs) out.push_back(val(t));
  return out;
}

int count_xor(const Slp &p) {
  int n = 0;
  for (const Stmt &s : p.stmts) n += (int)s.ops.size() - 1;
  return n;
}

int count_mem(const Slp &p) {
  int n = 0;
  for (const Stmt &s : p.stmts) n += (int)s.ops.size() + 1;
  return n;
}

int dfs_pebbles(const Slp &p) {
  // Pebble assignment of the DFS heuristic (Sec. 6.6): a statement takes a
  // movable pebble (its node no longer needed and not a goal) when there is
  // one, else a fresh pebble.  The count does not depend on which movable
  // pebble is taken.
  std::unordered_map<int, int> last_use;
  for (size_t i = 0; i < p.stmts.size(); ++i)
    for (int o : p.stmts[i].ops)
      if (!is_const(o) && o != kZero) last_use[o] = (int)i;
  std::set<int> goals;
  for (int o : p.outputs)
    if (!is_const(o) && o != kZero) goals.insert(o);
  int free_cnt = 0, npeb = 0;
  for (size_t i = 0; i < p.stmts.size(); ++i) {
    const Stmt &s = p.stmts[i];
    for (int o : s.ops)
      if (!is_const(o) && o != kZero && last_use[o] == (int)i && !goals.count(o)) ++free_cnt;
    if (free_cnt > 0) --free_cnt;
    else ++npeb;
    if (!goals.count(s.var) && !last_use.count(s.var)) ++free_cnt;
  }
  return npeb;
}

}  // namespace ec
