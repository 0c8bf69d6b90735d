// Continuous-batching server (placeholder until the server lands).
#include "pdiv_internal.hpp"

extern "C" {
pdiv_status pdiv_server_create(size_t, int32_t, pdiv_server* out) {
  if (out) *out = nullptr;
  return PDIV_ERR_UNSUPPORTED;
}
pdiv_status pdiv_server_put_field(pdiv_server, uint64_t, const void*, const void*, const void*,
                                  const void*, pdiv_dtype, int64_t, int64_t, double, double,
                                  uint64_t*) { return PDIV_ERR_UNSUPPORTED; }
pdiv_status pdiv_server_submit_lcp(pdiv_server, uint64_t, const float*, int32_t, float*,
                                   uint64_t*) { return PDIV_ERR_UNSUPPORTED; }
pdiv_status pdiv_server_wait(pdiv_server, uint64_t, int64_t, pdiv_status*) { return PDIV_ERR_UNSUPPORTED; }
pdiv_status pdiv_server_stats(pdiv_server, pdiv_server_stats_t*) { return PDIV_ERR_UNSUPPORTED; }
pdiv_status pdiv_server_destroy(pdiv_server) { return PDIV_ERR_UNSUPPORTED; }
}
