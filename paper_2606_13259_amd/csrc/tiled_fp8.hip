// Windowed VALU forward kernel instantiated for FP8 (E4M3) workspace storage
// (implementation and design notes in tiled_impl.h).
#include "tiled_impl.h"

namespace dasmi {
hipError_t tiled_forward_fp8(const Geom& g, const TileShape& ts, const Window& w, const void* ws,
                            int B, float* x, hipStream_t st) {
  return tiled::launch<uint8_t>(g, ts, w, ws, B, x, st);
}
size_t tiled_lds_fp8(const Geom& g, int bt, const Window& w) { return tiled::lds_bytes(g.Q, bt, w); }
hipError_t tiled_batched_fp8(const BatchedArgs& a, int bt, int qn, bool wtx, int cus,
                             hipStream_t st) {
  return tiled::launch_batched<uint8_t>(a, bt, qn, wtx, cus, st);
}
}  // namespace dasmi
