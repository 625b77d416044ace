// Windowed VALU forward kernel instantiated for f16 workspace storage
// (implementation and design notes in tiled_impl.h).
#include "tiled_impl.h"

namespace dasmi {
hipError_t tiled_forward_f16(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                            int B, float* x, hipStream_t st) {
  return tiled::launch<_Float16>(g, ts, w, ws, B, x, st);
}
size_t tiled_lds_f16(const Geom& g, int bt, const Window& w) { return tiled::lds_bytes(g.Q, bt, w); }
hipError_t tiled_batched_f16(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                             hipStream_t st) {
  return tiled::launch_batched<_Float16>(a, bt, qn, wtx, cus, st);
}
}  // namespace dasmi
