// Adjoint step: placeholder entry points until the adjoint kernels land.
#include "../../include/hard.h"
#include "api_internal.hpp"

using namespace hard;

extern "C" {
hard_status_t hard_adjoint_workspace_bytes(const hard_grid_t*, size_t*) {
  return fail(HARD_ERR_UNSUPPORTED, "adjoint step not built");
}
hard_status_t hard_hydro_step_adjoint(const hard_grid_t*, const void*, const double*, void*, void*, size_t, void*) {
  return fail(HARD_ERR_UNSUPPORTED, "adjoint step not built");
}
}
