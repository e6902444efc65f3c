// Tile-shape selection and the autotuner.
#include "dd_internal.h"

namespace dd {

TileShape shape_for(const dd_plan* plan, dd_dtype in_t, int64_t nsamp) {
  (void)nsamp;
  if (in_t == DD_F32) {
    TileShape s;
    s.variant = 1;  // register-window kernel, three waves per SIMD
    s.dms_per_wave = 8;
    s.waves = 4;
    s.tsamp_per_lane = 12;
    s.chans_per_stage = 8;
    return s;
  }
  return default_shape(in_t, plan);
}

}  // namespace dd

extern "C" dd_status dd_autotune(const dd_plan* plan, dd_dtype in_t, int64_t nsamp, void* stream,
                                 dd_tile_config* best, float* best_ms) {
  (void)plan; (void)in_t; (void)nsamp; (void)stream; (void)best; (void)best_ms;
  return dd::set_error(DD_ERR_NOT_IMPLEMENTED, "autotuner not built yet");
}
