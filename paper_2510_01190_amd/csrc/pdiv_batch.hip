// Batched persistent launch (placeholder until the batch kernel lands).
#include "pdiv_internal.hpp"

extern "C" {
pdiv_status pdiv_batch_create(const pdiv_field*, int32_t, pdiv_dtype, uint32_t, pdiv_stream,
                              pdiv_batch* out) {
  if (out) *out = nullptr;
  return PDIV_ERR_UNSUPPORTED;
}
pdiv_status pdiv_batch_launch(pdiv_batch, pdiv_stream) { return PDIV_ERR_UNSUPPORTED; }
pdiv_status pdiv_batch_info(pdiv_batch, int32_t*, int32_t*, int64_t*) { return PDIV_ERR_UNSUPPORTED; }
pdiv_status pdiv_batch_destroy(pdiv_batch) { return PDIV_ERR_UNSUPPORTED; }
}
