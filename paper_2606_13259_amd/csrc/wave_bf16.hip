// Wavefront-tiled VALU forward kernel instantiated for bf16 workspace storage
// (implementation and design notes in wave_impl.h).
#include "wave_impl.h"

namespace dasmi {
hipError_t wave_forward_bf16(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                           int B, float* x, hipStream_t st) {
  const wavek::BoxShape bs{ts.tx, ts.ty, ts.tz, ts.lx, ts.lxy};
  return wavek::launch<uint16_t>(g, bs, w, ws, B, x, st);
}
}  // namespace dasmi
