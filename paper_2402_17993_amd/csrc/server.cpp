// Continuous-batching VQE server (include/ucc.h, "serving").
#include "api_internal.h"

using namespace ucc;

extern "C" {

ucc_status ucc_server_create(size_t, int32_t, int32_t, ucc_server** out) {
  if (out) *out = nullptr;
  return fail(UCC_EINVAL, "server not available in this build");
}
ucc_status ucc_submit(ucc_server*, ucc_ctx*, const double*, int32_t, double, uint32_t, uint64_t*) {
  return fail(UCC_EINVAL, "server not available in this build");
}
ucc_status ucc_poll(ucc_server*, uint64_t, int32_t*, double*, double*, double*) {
  return fail(UCC_EINVAL, "server not available in this build");
}
ucc_status ucc_wait(ucc_server*, uint64_t, double*, double*, double*) {
  return fail(UCC_EINVAL, "server not available in this build");
}
ucc_status ucc_cancel(ucc_server*, uint64_t) {
  return fail(UCC_EINVAL, "server not available in this build");
}
void ucc_server_destroy(ucc_server*) {}

}  // extern "C"
