// Windowed VALU forward for complex baseband (IQ) data with f32 workspace
// storage: batch items come in (I, Q) pairs and every term is remodulated by
// exp(i 2 pi fc tau) (implementation in tiled_impl.h).
#include "tiled_impl.h"

namespace dasmi {
hipError_t tiled_forward_f32_iq(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                                int B, float* x, hipStream_t st) {
  return tiled::launch_iq<float>(g, ts, w, ws, B, x, st);
}
}  // namespace dasmi
