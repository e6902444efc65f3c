// Streaming server with continuous batching.
#include "dd_internal.h"

extern "C" {
dd_status dd_serve_create(const dd_serve_config*, void*, size_t, dd_server**) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "serving not built yet");
}
dd_status dd_serve_add_beam(dd_server*, const dd_plan*, int64_t, int32_t*) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "serving not built yet");
}
dd_status dd_serve_submit(dd_server*, int32_t, const void*, int64_t, int64_t, uint64_t*) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "serving not built yet");
}
dd_status dd_serve_poll(dd_server*, dd_result*, int32_t, int32_t*) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "serving not built yet");
}
dd_status dd_serve_release(dd_server*, uint64_t) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "serving not built yet");
}
dd_status dd_serve_drain(dd_server*) {
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "serving not built yet");
}
dd_status dd_serve_destroy(dd_server*) { return DD_OK; }
}
