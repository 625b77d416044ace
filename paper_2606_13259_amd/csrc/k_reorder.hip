// Channel-data reorder + precision conversion (paper, Sec. 3.2 and Sec. 3.3):
// y[nb][Q][M][K] f32  ->  ws[Q][M][K][btot] (items b0 .. b0+nb-1), stored as
// f32, f16 or bf16 (round to nearest even).  Batch-inner order makes the items
// that one lane group reads at a given (q, m, k) contiguous.
//
// HBM-bound: per element 4 bytes read and 2 or 4 bytes written.
#include "das_device.h"

namespace dasmi {
namespace {

__device__ inline void store_cvt(float* p, float v) { *p = v; }
__device__ inline void store_cvt(_Float16* p, float v) { *p = (_Float16)v; }
__device__ inline void store_cvt(uint16_t* p, float v) {
  // f32 -> bf16, round to nearest even; NaN stays NaN (quiet bit set).
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    *p = (uint16_t)((u >> 16) | 0x40u);
    return;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  *p = (uint16_t)(u >> 16);
}

// nb == 1 (and the copy for the plain layout): a streaming convert-copy,
// four elements per lane per step.
template <class T>
__global__ __launch_bounds__(256) void copy_convert(const float* __restrict__ y, size_t n,
                                                    T* __restrict__ out, size_t out_stride,
                                                    size_t out_off) {
  const size_t stride = (size_t)gridDim.x * blockDim.x * 4;
  for (size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    if (i + 4 <= n) {
      const float4 v = *reinterpret_cast<const float4*>(y + i);
      store_cvt(out + (i + 0) * out_stride + out_off, v.x);
      store_cvt(out + (i + 1) * out_stride + out_off, v.y);
      store_cvt(out + (i + 2) * out_stride + out_off, v.z);
      store_cvt(out + (i + 3) * out_stride + out_off, v.w);
    } else {
      for (size_t j = i; j < n; ++j) store_cvt(out + j * out_stride + out_off, y[j]);
    }
  }
}

// nb >= 2: transpose through LDS, 64 positions (q, m, k flattened) x up to 64
// batch items per block.
template <class T>
__global__ __launch_bounds__(256) void transpose_convert(const float* __restrict__ y, long long nqmk,
                                                         int nb, int b0, int btot,
                                                         T* __restrict__ ws) {
  __shared__ float tile[64][65];
  const int t = threadIdx.x;
  const long long i0 = (long long)blockIdx.x * 64;
  const int bb0 = blockIdx.y * 64;
  const int nbc = min(64, nb - bb0);
  {
    const int il = t & 63;
    const long long i = i0 + il;
    for (int bl = t >> 6; bl < nbc; bl += 4)
      tile[bl][il] = (i < nqmk) ? y[(long long)(bb0 + bl) * nqmk + i] : 0.f;
  }
  __syncthreads();
  const int rows = 256 / nbc;  // i-rows written per pass
  const int row0 = t / nbc, bl = t - row0 * nbc;
  if (row0 < rows) {
    for (int il = row0; il < 64; il += rows) {
      const long long i = i0 + il;
      if (i < nqmk) store_cvt(ws + i * btot + b0 + bb0 + bl, tile[bl][il]);
    }
  }
}

template <class T>
hipError_t reorder_t(const Geom& g, const float* y, int b0, int nb, int btot, void* ws,
                     hipStream_t st) {
  const long long nqmk = (long long)g.Q * g.M * g.K;
  T* out = static_cast<T*>(ws);
  if (nb == 1 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    const size_t blocks = (size_t)std::min<long long>((nqmk / 4 + 255) / 256 + 1, 65536);
    hipLaunchKernelGGL(copy_convert<T>, dim3((unsigned)blocks), dim3(256), 0, st, y,
                       (size_t)nqmk, out, (size_t)btot, (size_t)b0);
  } else {
    dim3 grid((unsigned)((nqmk + 63) / 64), (unsigned)((nb + 63) / 64));
    hipLaunchKernelGGL(transpose_convert<T>, grid, dim3(256), 0, st, y, nqmk, nb, b0, btot, out);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reorder(const Geom& g, int storage, const float* y, int b0, int nb, int btot,
                          void* ws, hipStream_t st) {
  switch (storage) {
    case DAS_STORE_F32: return reorder_t<float>(g, y, b0, nb, btot, ws, st);
    case DAS_STORE_F16: return reorder_t<_Float16>(g, y, b0, nb, btot, ws, st);
    default: return reorder_t<uint16_t>(g, y, b0, nb, btot, ws, st);
  }
}

}  // namespace dasmi
