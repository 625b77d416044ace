// Wavefront-tiled VALU forward kernel instantiated for f16 workspace storage
// (implementation and design notes in wave_impl.h).
#include "wave_impl.h"

namespace dasmi {
hipError_t wave_forward_f16(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                           int B, float* x, hipStream_t st) {
  const wavek::BoxShape bs{ts.tx, ts.ty, ts.tz, ts.lx, ts.lxy};
  return wavek::launch<_Float16>(g, bs, w, ws, B, x, st);
}
}  // namespace dasmi
