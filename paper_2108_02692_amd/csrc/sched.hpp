// sched.hpp -- register-slot allocation and bytecode emission.
#pragma once

#include <cstdint>
#include <vector>

#include "slp.hpp"

namespace ec {

struct SchedOpts {
  int slots = 32;  // register slots (16 B per lane each)
  int hoist = 24;  // max program ops a load is issued ahead of its first read
  int max_inflight = 48;  // cap on outstanding vector memory operations
};

struct SchedResult {
  std::vector<uint32_t> words;
  int slots_used = 0;
  int peak_live = 0;
  int n_loads = 0;
  int n_stores = 0;
};

// Allocates the program's values to `opts.slots` register slots and emits
// the per-tile bytecode.  Returns 0, or -1 when live temporaries alone
// exceed the slot budget.
int schedule(const Slp &p, int n_in_strips, int n_out_strips, const SchedOpts &opts, SchedResult &out);

// Broadcast form of the plain bitmatrix program: output rows accumulate in
// slots 0..R-1; every input strip is loaded once into a ring of prefetch
// slots, pulled into the accumulator and pushed into each row whose
// bitmatrix entry is 1.  Returns 0, or -1 when fewer than 2 slots remain for
// the ring.
int schedule_broadcast(const std::vector<Bits> &rows, int n_in_strips, const SchedOpts &opts, SchedResult &out);

// Structural check of a bytecode stream against its limits: every slot below
// `slots`, every strip in range, WAIT counts valid, terminated by HALT.
bool validate_bytecode(const std::vector<uint32_t> &w, int slots, int n_in_strips, int n_out_strips);

}  // namespace ec
