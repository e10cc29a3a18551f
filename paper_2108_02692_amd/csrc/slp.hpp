// slp.hpp -- XOR straight-line programs and the paper's transformations.
//
// Terms are ints: variables are >= 0 and < kConstBase; input array (strip) c
// is kConstBase + c; kZero is the all-zero array.  A program is a list of
// statements var <- XOR(ops...) and one returned term per output strip
// (Sec. 4.1; multi-input statements are the MultiSLP of Sec. 5.1).
#pragma once

#include <cstdint>
#include <vector>

#include "gf.hpp"

namespace ec {

constexpr int kZero = -1;
constexpr int kConstBase = 1 << 20;
inline bool is_const(int t) { return t >= kConstBase; }

// Set of input strips (up to 256 = 32 blocks x 8 strips), the value of a
// term under the set semantics of Sec. 4.1 (XOR = symmetric difference).
struct Bits {
  uint64_t w[4] = {0, 0, 0, 0};
  void flip(int i) { w[i >> 6] ^= 1ull << (i & 63); }
  bool test(int i) const { return (w[i >> 6] >> (i & 63)) & 1u; }
  int count() const {
    return __builtin_popcountll(w[0]) + __builtin_popcountll(w[1]) + __builtin_popcountll(w[2]) +
           __builtin_popcountll(w[3]);
  }
  Bits operator^(const Bits &o) const {
    Bits r;
    for (int k = 0; k < 4; ++k) r.w[k] = w[k] ^ o.w[k];
    return r;
  }
  bool operator==(const Bits &o) const {
    return w[0] == o.w[0] && w[1] == o.w[1] && w[2] == o.w[2] && w[3] == o.w[3];
  }
};

struct Stmt {
  int var;
  std::vector<int> ops;
};

struct Slp {
  int n_const = 0;
  std::vector<Stmt> stmts;
  std::vector<int> outputs;
};

// Bitmatrix (Sec. 1): row 8*i+r of the expansion of a rows x cols GF(2^8)
// matrix, as the set of columns 8*j+c whose bit is 1, where the 8x8 block of
// element e has column c = bits of e * x^c.
std::vector<Bits> bitmatrix_rows(int rows, int cols, const Mat &m);

// Plain program: one statement per bit row over its input strips (Sec. 2).
Slp plain_slp(const std::vector<Bits> &rows, int n_const);

// RePair (Sec. 4.3), or XorRePair (Sec. 4.4) when `rebuild` is set.
Slp xor_repair(const std::vector<Bits> &rows, int n_const, bool rebuild);

// XOR fusion (Sec. 5.2).
Slp fuse(const Slp &in);

// DFS post-order over the computation graph (Sec. 6.6), from the returned
// variables in their order, then from any other statement no statement uses.
Slp dfs_schedule(const Slp &in);

// Bottom-up greedy heuristic (Sec. 6.6) for an LRU cache of `capacity`
// entries.  The result assigns pebbles: every statement's var is a pebble
// number (pebbles are reassigned), operands name pebbles or constants, and
// the outputs name the pebbles holding the returned values at the end.
Slp greedy_schedule(const Slp &in, int capacity);

// Set-semantics value of every returned term.
std::vector<Bits> evaluate(const Slp &p);

// Measures (Secs. 4.1, 5.1, 6.6).
int count_xor(const Slp &p);   // sum (arity - 1)
int count_mem(const Slp &p);   // sum (arity + 1)
int dfs_pebbles(const Slp &p); // pebbles of the DFS assignment (NVar after scheduling)

}  // namespace ec
