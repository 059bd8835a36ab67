// Batched form (persistent kernel over many instances).  Placeholder until the persistent
// kernel lands: every entry point reports IDW_EUNSUPPORTED.
#include <hip/hip_runtime.h>

#include "../../include/idw.h"
#include "idw_api_internal.hpp"

using namespace idw;

extern "C" {

int idw_batched_plan_create(const idw_instance*, int32_t, int32_t, const idw_config*, idw_plan** out) {
  clear_error();
  if (out) *out = nullptr;
  return fail(IDW_EUNSUPPORTED, "batched plans are not available in this build");
}

int idw_batched_plan_workspace(const idw_plan*, size_t* bytes) {
  clear_error();
  if (bytes) *bytes = 0;
  return fail(IDW_EUNSUPPORTED, "batched plans are not available in this build");
}

int idw_batched(idw_plan*, void*, size_t, void*) {
  clear_error();
  return fail(IDW_EUNSUPPORTED, "batched plans are not available in this build");
}

void idw_batched_plan_destroy(idw_plan*) {}

}  // extern "C"
