// program_pool.hpp -- device memory for compiled programs' records.
//
// Every program's device image (its records and those of its parts) lives
// in a per-device pool: chunks of device memory, each handed out first-fit,
// with identical images stored once (looked up by a hash of their words and
// compared in full).  A program takes a reference on first use on a device
// and drops it when freed; chunks stay allocated for the process's
// lifetime.  reserve() sizes a chunk for many programs at once, so that
// uploading a whole set of programs makes one allocation.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/ec.h"

namespace ec {

// Device copy of `image` on device `dev` (the current device), shared with
// any identical image already there; nullptr and *st set on failure
// (EC_ERR_NOMEM, EC_ERR_DEVICE).
const uint32_t *pool_acquire(int dev, const std::vector<uint32_t> &image, ec_status *st);

// Drops one reference to a copy returned by pool_acquire; its space is
// reused once no program refers to it.  Makes no HIP call.
void pool_release(int dev, const uint32_t *words);

// Bytes that placing all of `images` on device `dev` would take beyond what
// is there (each distinct image not yet in the pool, rounded to the pool's
// placement granule).
size_t pool_missing_bytes(int dev, const std::vector<const std::vector<uint32_t> *> &images);

// Makes sure one chunk on device `dev` has `bytes` free in one piece (at most
// one allocation).
ec_status pool_reserve(int dev, size_t bytes);

// Chunks allocated, images held and bytes in use on device `dev`.
void pool_stats(int dev, int *chunks, int *images, size_t *bytes_used);

}  // namespace ec
