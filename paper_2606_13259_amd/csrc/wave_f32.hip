// Wavefront-tiled VALU forward kernel instantiated for f32 workspace storage
// (implementation and design notes in wave_impl.h).
#include "wave_impl.h"

namespace dasmi {
hipError_t wave_forward_f32(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                           int B, float* x, hipStream_t st) {
  const wavek::BoxShape bs{ts.tx, ts.ty, ts.tz, ts.lx, ts.lxy};
  return wavek::launch<float>(g, bs, w, ws, B, x, st);
}
}  // namespace dasmi
