// Entry points whose kernels are not in this build yet: they return
// TSSPGEMM_ERR_UNSUPPORTED with a message.
#include "api_internal.hpp"

using namespace tss;

extern "C" {

int tsspgemm_batched_plan(int32_t, const tsspgemm_csr*, const tsspgemm_csr*, const tsspgemm_tuning*, tsspgemm_batch*,
                          int64_t*, int64_t*, void*) {
  set_error("tsspgemm_batched_plan: not available in this build");
  return TSSPGEMM_ERR_UNSUPPORTED;
}
int tsspgemm_batched_run(tsspgemm_batch, int32_t*, int32_t*, float*, int64_t*, void*) {
  set_error("tsspgemm_batched_run: not available in this build");
  return TSSPGEMM_ERR_UNSUPPORTED;
}
void tsspgemm_batched_destroy(tsspgemm_batch) {}

}  // extern "C"
