// Tile-shape selection and the autotuner.
#include "dd_internal.h"

namespace dd {

TileShape shape_for(const dd_plan* plan, dd_dtype in_t, int64_t nsamp) {
  (void)nsamp;
  return default_shape(in_t, plan);
}

}  // namespace dd

extern "C" dd_status dd_autotune(const dd_plan* plan, dd_dtype in_t, int64_t nsamp, void* stream,
                                 dd_tile_config* best, float* best_ms) {
  (void)plan; (void)in_t; (void)nsamp; (void)stream; (void)best; (void)best_ms;
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "autotuner not built yet");
}
