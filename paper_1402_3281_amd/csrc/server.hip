// server.hip -- served partition jobs (continuous batching).
#include <hip/hip_runtime.h>

#include "engine.h"

using namespace sclap;

extern "C" {

int sclap_server_create(sclap_ctx*, int64_t, int32_t, sclap_server** out) {
  if (out) *out = nullptr;
  return fail(SCLAP_EINVAL, "server not available in this build");
}
int sclap_server_submit(sclap_server*, const sclap_job*, uint64_t*) { return fail(SCLAP_EINVAL, "no server"); }
int sclap_server_poll(sclap_server*, uint64_t, sclap_job_result*) { return fail(SCLAP_EINVAL, "no server"); }
int sclap_server_wait(sclap_server*, uint64_t, sclap_job_result*) { return fail(SCLAP_EINVAL, "no server"); }
int sclap_server_stats(sclap_server*, double*, double*, double*, int64_t*, int64_t*) {
  return fail(SCLAP_EINVAL, "no server");
}
int sclap_server_destroy(sclap_server*) { return SCLAP_OK; }
}
