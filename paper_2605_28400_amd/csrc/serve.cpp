// Serving entry points (continuous batching). Placeholder until the server
// runtime lands: every call reports that serving is unavailable.
#include "common.h"

using namespace trioseq;

extern "C" {
trioseq_status trioseq_serve_create(const trioseq_serve_config*, const trioseq_scoring*,
                                    trioseq_server**) {
  return fail(TRIOSEQ_ERR_INVALID_ARG, "serving is not available in this build");
}
trioseq_status trioseq_serve_submit(trioseq_server*, const trioseq_triplet*, uint64_t*) {
  return fail(TRIOSEQ_ERR_INVALID_ARG, "serving is not available in this build");
}
trioseq_status trioseq_serve_poll(trioseq_server*, trioseq_result*, size_t, size_t*) {
  return fail(TRIOSEQ_ERR_INVALID_ARG, "serving is not available in this build");
}
trioseq_status trioseq_serve_wait(trioseq_server*, uint64_t, trioseq_result*, int64_t) {
  return fail(TRIOSEQ_ERR_INVALID_ARG, "serving is not available in this build");
}
trioseq_status trioseq_serve_get_stats(trioseq_server*, trioseq_serve_stats*) {
  return fail(TRIOSEQ_ERR_INVALID_ARG, "serving is not available in this build");
}
trioseq_status trioseq_serve_destroy(trioseq_server*) {
  return fail(TRIOSEQ_ERR_INVALID_ARG, "serving is not available in this build");
}
}
