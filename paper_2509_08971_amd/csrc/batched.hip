// Batched step: placeholder entry points until the batched kernels land.
#include "../../include/hard.h"
#include "api_internal.hpp"

using namespace hard;

extern "C" {
hard_status_t hard_batch_plan_create(const hard_grid_t*, int32_t, const char*, hard_batch_plan_t** out) {
  if (out) *out = nullptr;
  return fail(HARD_ERR_UNSUPPORTED, "batched step not built");
}
hard_status_t hard_batch_plan_destroy(hard_batch_plan_t*) { return ok(); }
hard_status_t hard_batch_offsets(const hard_batch_plan_t*, int64_t*) {
  return fail(HARD_ERR_UNSUPPORTED, "batched step not built");
}
hard_status_t hard_batch_workspace_bytes(const hard_batch_plan_t*, size_t*) {
  return fail(HARD_ERR_UNSUPPORTED, "batched step not built");
}
hard_status_t hard_cfl_dt_batched(const hard_batch_plan_t*, const void*, double, double*, void*, size_t, void*) {
  return fail(HARD_ERR_UNSUPPORTED, "batched step not built");
}
hard_status_t hard_hydro_step_batched(const hard_batch_plan_t*, void*, double*, double, int32_t, void*, size_t, void*) {
  return fail(HARD_ERR_UNSUPPORTED, "batched step not built");
}
}
