// push.hpp -- programs in push form and their register-slot schedule.
//
// The executor evaluates a program value by value: a value (an input strip
// or a finished temporary) is brought into the accumulator once and XORed
// into every accumulator slot that consumes it.  Output rows are
// accumulators for the whole tile; temporaries are accumulators from their
// first incoming value until they are complete.  This is the multi-input
// XOR of Sec. 5.1 evaluated in the order its inputs arrive, with registers
// as the only storage (no temporary reaches memory, Sec. 5).
#pragma once

#include <cstdint>
#include <vector>

#include "slp.hpp"

namespace ec {

// Accumulators 0..n_rows-1 are the output rows, the rest temporaries.
// src[a] lists the values XORed into accumulator a: an input strip
// (kConstBase + c) or a temporary (its accumulator index).  `order` is the
// order in which input strips are brought in.
struct PushDag {
  int n_const = 0;
  int n_rows = 0;
  std::vector<std::vector<int>> src;
  std::vector<int> order;
};

// Plain bitmatrix program: row r's sources are the strips of its 1 bits.
PushDag push_plain(const std::vector<Bits> &rows, int n_const);

// Column-blocked compression: the bitmatrix is cut into column blocks of
// `width` strips (one data block when width = 8); every block's slice is
// compressed by RePair / XorRePair (Secs. 4.3-4.4) and, with `fused`, fused
// (Sec. 5.2).  Each block's program only reads that block's strips, so its
// temporaries live while its strips are brought in and the register file
// bounds them.  `blocks`, when given, receives the per-block programs (local
// strip numbering) for inspection.
PushDag push_blocked(const std::vector<Bits> &rows, int n_const, int width, bool rebuild, bool fused,
                     std::vector<Slp> *blocks = nullptr);

// Push-form unfolding: a temporary with a sources and k consumers costs
// about a + k slot XORs plus one record, against a * k XORs when its sources
// are pushed into every consumer directly; temporaries with
// a * k <= a + k + record_cost are inlined (repeatedly, cheapest first).
void push_unfold(PushDag &d, int record_cost);

// Orders the strips inside every column block greedily so that as few
// temporaries as possible are open at once (ties: more completed, then the
// lower strip).
void push_order(PushDag &d, int width);

// Orders the strips by the bottom-up greedy heuristic of Sec. 6.6: the
// program in statement form (push_as_slp) is scheduled for an LRU cache of
// `capacity` entries (the register slots), and the strips are brought in in
// the order that schedule first reads them.  With width > 0 the column
// blocks keep their order (a temporary combines strips of one block only, so
// interleaving blocks would only hold temporaries open longer) and the
// greedy order applies within each block.
void push_order_greedy(PushDag &d, int width, int capacity);

// Set-semantics value of every row.
std::vector<Bits> push_eval(const PushDag &d);

// The push program as a straight-line program: temporaries in completion
// order, then one statement per row.
Slp push_as_slp(const PushDag &d);

struct PushOpts {
  int slots = 40;     // register slots (16 B per lane each)
  int max_ring = 12;  // most input strips loaded ahead of their use
  int prefetch = 0;   // strips touched this far ahead of their register load (0 = none)
  int row_lo = 0;     // rows scheduled: [row_lo, row_hi) (whole output blocks
  int row_hi = -1;    // or any run of rows; -1: every row)
};

struct PushCode {
  std::vector<uint32_t> words;
  int slots_used = 0;
  int peak_open = 0;  // temporaries open at once
  int ring = 0;       // input strips loaded ahead
  int passes = 0;     // passes over the inputs (more than one only when the rows do not fit)
  int n_loads = 0;
  int n_stores = 0;
  int n_prefetch = 0;
  int n_records = 0;
  int n_ops = 0;      // run operands (slot XORs) per tile
};

// Schedules `d` on `opts.slots` slots for a stripe whose input blocks are
// table entries 0..n_in_blocks-1 and output rows go to entries n_in_blocks..
// (row r: entry n_in_blocks + r / 8, strip r % 8).  Returns 0, or -1 when not
// even one output block's rows fit beside its open temporaries.
int push_schedule(const PushDag &d, int n_in_blocks, const PushOpts &opts, PushCode &out);

// Structural check of a record stream: fields in range, unused bits zero,
// operands and slots below `slots`, blocks inside the table, HALT followed
// by a zero window.
bool validate_code(const std::vector<uint32_t> &w, int slots, int n_in_blocks, int n_out_blocks);

// Runs a record stream on set-valued slots for two consecutive tiles (from
// all-zero slots; the second tile starts from the state the first leaves)
// and checks that every output strip of both equals `rows`, that no slot is
// read before its load has been waited for, that no load lands in a slot
// that is still being read or accumulated, and that every slot is zero again
// at the end of a tile.
// With row_lo / row_hi, only rows [row_lo, row_hi) are expected, and a
// store of any other row is an error.
bool simulate_code(const std::vector<uint32_t> &w, int slots, int n_in_blocks, int n_out_blocks,
                   const std::vector<Bits> &rows, int row_lo = 0, int row_hi = -1);

}  // namespace ec
