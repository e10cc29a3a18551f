// batch.hpp -- planning of a multi-stripe launch, shared by the batch
// objects (batch.cpp) and the entry point that allocates nothing
// (noalloc.hip).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/ec.h"
#include "exec.hpp"

namespace ec {

// A byte range [first, second) read or written by a launch.
struct ByteRange {
  uintptr_t first, second;
};

// What a set of stripes needs: validated, with the row split decided for the
// whole batch and the table sizes counted.
struct BatchPlan {
  int slots = 0;                 // the programs' common slot budget
  uint32_t tiles_per_item = 1;   // tiles one work item covers
  size_t in_bytes = 0, out_bytes = 0;
  size_t n_ranges_in = 0, n_ranges_out = 0;  // input and output blocks over all stripes
  uint64_t n_items = 0;          // work items (two words each)
  bool rows_fit = false, pairs_fit = false, blocks_fit = false;  // the split of EC_SPLIT_AUTO stripes
};

// Validates the stripes (pointers, sizes, alignment, one slot budget) and
// decides the row split for a device of n_cus compute units.  Writes nothing
// but *plan.  Errors as ec_batch_set (except the overlap check, see
// batch_fill).
ec_status batch_plan(const ec_stripe *stripes, int n_stripes, size_t tile_bytes, int n_cus, BatchPlan *plan);

// Writes the n_stripes descriptors and the 2 * plan.n_items item words for
// device `dev` (the current device), and, when reads and writes are given
// (workspaces of plan.n_ranges_in / plan.n_ranges_out entries), checks that
// no output block overlaps another output block or any input block.
// upload = true copies a program to the device if it is not there yet (an
// allocation); false makes such a program an EC_ERR_ARG.
ec_status batch_fill(const ec_stripe *stripes, int n_stripes, const BatchPlan &plan, int dev, bool upload,
                     StripeDesc *desc, uint32_t *items, ByteRange *reads, ByteRange *writes);

// Workgroups of the persistent kernel for a plan on a device of n_cus CUs.
int batch_grid(const BatchPlan &plan, int n_cus);

// ec_batch_set; check_overlap = false skips the check that outputs overlap
// no other output and no input (for a caller whose buffers are disjoint by
// construction, such as the serving loop with its output arena).
ec_status batch_set(ec_batch *b, const ec_stripe *stripes, int n_stripes, size_t tile_bytes, ec_stream stream,
                    bool check_overlap);

}  // namespace ec
