// Entry points whose kernels are not in this build yet: they return
// TSSPGEMM_ERR_UNSUPPORTED with a message.
#include "api_internal.hpp"

using namespace tss;

extern "C" {

int tsspgemm_msbfs(const tsspgemm_csr*, const int32_t*, int32_t, int32_t*, int32_t*, int64_t*, int32_t, void*) {
  set_error("tsspgemm_msbfs: not available in this build");
  return TSSPGEMM_ERR_UNSUPPORTED;
}
int tsspgemm_transpose(const tsspgemm_csr*, int32_t*, int32_t*, int32_t*, void*) {
  set_error("tsspgemm_transpose: not available in this build");
  return TSSPGEMM_ERR_UNSUPPORTED;
}
int tsspgemm_grad_a(tsspgemm_plan, const tsspgemm_csr*, const tsspgemm_csr*, const tsspgemm_csr*, float*, void*) {
  set_error("tsspgemm_grad_a: not available in this build");
  return TSSPGEMM_ERR_UNSUPPORTED;
}
int tsspgemm_grad_b(tsspgemm_plan, const tsspgemm_csr*, const int32_t*, const tsspgemm_csr*, const tsspgemm_csr*,
                    const tsspgemm_csr*, float*, void*) {
  set_error("tsspgemm_grad_b: not available in this build");
  return TSSPGEMM_ERR_UNSUPPORTED;
}
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
