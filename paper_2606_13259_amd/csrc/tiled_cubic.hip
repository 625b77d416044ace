// Windowed VALU forward with four-point Lagrange (cubic) interpolation and f32
// workspace storage (implementation in tiled_impl.h).
#include "tiled_impl.h"

namespace dasmi {
hipError_t tiled_forward_f32_cubic(const Geom& g, const TileShape& ts, const Window& w,
                                   const void* ws, int B, float* x, hipStream_t st) {
  return tiled::launch_cubic<float>(g, ts, w, ws, B, x, st);
}
}  // namespace dasmi
