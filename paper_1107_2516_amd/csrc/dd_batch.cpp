// Batched many-beam execution.
#include "dd_internal.h"

extern "C" {
dd_status dd_batch_create(const dd_batch_item*, int32_t, dd_dtype, dd_dtype, dd_batch**) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "batching not built yet");
}
dd_status dd_batch_update(dd_batch*, const dd_batch_item*, int32_t) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "batching not built yet");
}
dd_status dd_batch_launch(dd_batch*, void*) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "batching not built yet");
}
dd_status dd_batch_destroy(dd_batch*) { return DD_OK; }
}
