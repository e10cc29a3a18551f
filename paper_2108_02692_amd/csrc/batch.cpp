// batch.cpp -- multi-stripe launches (filled in with the persistent kernel).
#include "../../include/ec.h"

extern "C" {

ec_status ec_batch_build(const ec_stripe *, int, size_t, ec_stream, ec_batch **out) {
  if (out) *out = nullptr;
  return EC_ERR_UNSUPPORTED;
}
ec_status ec_batch_launch(ec_batch *, ec_stream) { return EC_ERR_UNSUPPORTED; }
ec_status ec_batch_query(const ec_batch *, size_t *, size_t *, size_t *) { return EC_ERR_UNSUPPORTED; }
void ec_batch_free(ec_batch *) {}

}  // extern "C"
