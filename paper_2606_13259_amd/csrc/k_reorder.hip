// Channel-data reorder + precision conversion (paper, Sec. 3.2 and Sec. 3.3):
// y[nb][Q][M][K] f32  ->  ws[Q][M][K][btot] (items b0 .. b0+nb-1), stored as
// f32, f16, bf16 or FP8 E4M3 (round to nearest even; FP8 with the item's
// power-of-two scale).  Batch-inner order makes the items that one lane group
// reads at a given (q, m, k) contiguous.
//
// HBM-bound: per element 4 bytes read and 1, 2 or 4 bytes written (FP8 reads
// y twice: once for the largest magnitude of each item).
#include "das_device.h"
#include "fp8.h"

namespace dasmi {
namespace {


__device__ inline void store_cvt(float* p, float v, int) { *p = v; }
__device__ inline void store_cvt(_Float16* p, float v, int) { *p = (_Float16)v; }
__device__ inline void store_cvt(uint8_t* p, float v, int e) { *p = (uint8_t)e4m3_bits(ldexpf(v, e)); }
__device__ inline void store_cvt(uint16_t* p, float v, int) {
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
// FP8 stores item b as y 2^e with e = fp8_item_exponent(amax[b]); the other
// storage types pass amax = nullptr and ignore it.
template <class T>
__device__ inline int item_exponent(const float* amax, int b) {
  if constexpr (__is_same(T, uint8_t)) return fp8_item_exponent(amax[b]);
  return 0;
}

template <class T>
__global__ __launch_bounds__(256) void copy_convert(const float* __restrict__ y, size_t n,
                                                    T* __restrict__ out, size_t out_stride,
                                                    size_t out_off, const float* __restrict__ amax) {
  const int e = item_exponent<T>(amax, (int)out_off);
  const size_t stride = (size_t)gridDim.x * blockDim.x * 4;
  for (size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    if (i + 4 <= n) {
      const float4 v = *reinterpret_cast<const float4*>(y + i);
      store_cvt(out + (i + 0) * out_stride + out_off, v.x, e);
      store_cvt(out + (i + 1) * out_stride + out_off, v.y, e);
      store_cvt(out + (i + 2) * out_stride + out_off, v.z, e);
      store_cvt(out + (i + 3) * out_stride + out_off, v.w, e);
    } else {
      for (size_t j = i; j < n; ++j) store_cvt(out + j * out_stride + out_off, y[j], e);
    }
  }
}

// Contiguous output (one item: ws has the layout of y): each thread moves
// four 16-byte loads of four samples each, all issued before the first
// conversion, and writes each group of four converted samples with one
// vector store (16, 8 or 4 bytes).
template <class T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<_Float16> { using type = uint2; };
template <> struct Vec4<uint16_t> { using type = uint2; };
template <> struct Vec4<uint8_t> { using type = uint32_t; };

template <class T>
__device__ inline typename Vec4<T>::type cvt4(float4 v, int e) {
  if constexpr (__is_same(T, float)) {
    return v;
  } else if constexpr (__is_same(T, uint8_t)) {
    return e4m3_bits(ldexpf(v.x, e)) | (e4m3_bits(ldexpf(v.y, e)) << 8) |
           (e4m3_bits(ldexpf(v.z, e)) << 16) | ((uint32_t)e4m3_bits(ldexpf(v.w, e)) << 24);
  } else {
    T h[4];
    store_cvt(&h[0], v.x, e);
    store_cvt(&h[1], v.y, e);
    store_cvt(&h[2], v.z, e);
    store_cvt(&h[3], v.w, e);
    uint2 r;
    __builtin_memcpy(&r, h, sizeof(r));
    return r;
  }
}

constexpr int kCopyUnroll = 4;
template <class T>
__global__ __launch_bounds__(256) void copy_convert_contig(const float* __restrict__ y, size_t n4,
                                                           T* __restrict__ out,
                                                           const float* __restrict__ amax, int item) {
  using V = typename Vec4<T>::type;
  const int e = item_exponent<T>(amax, item);
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4* src = reinterpret_cast<const f4*>(y);
  V* dst = reinterpret_cast<V*>(out);
  const size_t per_block = (size_t)blockDim.x * kCopyUnroll;
  const size_t base = (size_t)blockIdx.x * per_block + threadIdx.x;
  float4 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const size_t i = base + (size_t)u * blockDim.x;
    f4 w = {0.f, 0.f, 0.f, 0.f};
    if (i < n4) w = __builtin_nontemporal_load(src + i);
    v[u] = float4{w.x, w.y, w.z, w.w};
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const size_t i = base + (size_t)u * blockDim.x;
    if (i < n4) dst[i] = cvt4<T>(v[u], e);
  }
}

// nb >= 2: transpose through LDS, 64 positions (q, m, k flattened) x up to 64
// batch items per block.
template <class T>
__global__ __launch_bounds__(256) void transpose_convert(const float* __restrict__ y, long long nqmk,
                                                         int nb, int b0, int btot,
                                                         T* __restrict__ ws,
                                                         const float* __restrict__ amax) {
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
    const int e = item_exponent<T>(amax, b0 + bb0 + bl);
    for (int il = row0; il < 64; il += rows) {
      const long long i = i0 + il;
      if (i < nqmk) store_cvt(ws + i * btot + b0 + bb0 + bl, tile[bl][il], e);
    }
  }
}

__global__ void zero_items(unsigned* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Largest |y| of each item: the bits of |y| order like the values (NaN above
// +inf), so a block keeps an integer maximum and merges it with one atomicMax.
// Grid: (blocks over one item, items); n elements per item, nb items.
__global__ __launch_bounds__(256) void item_absmax(const float* __restrict__ y, long long n, int nb,
                                                   unsigned* __restrict__ amax_bits) {
  __shared__ unsigned part[4];
  for (int b = blockIdx.y; b < nb; b += gridDim.y) {
    const float* yb = y + (long long)b * n;
    unsigned m = 0u;
    const long long stride = (long long)gridDim.x * blockDim.x * 4;
    const bool vec = (reinterpret_cast<uintptr_t>(yb) & 15) == 0;
    for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
      if (vec && i + 4 <= n) {
        const float4 v = *reinterpret_cast<const float4*>(yb + i);
        m = max(m, max(max(__float_as_uint(v.x) & 0x7fffffffu, __float_as_uint(v.y) & 0x7fffffffu),
                       max(__float_as_uint(v.z) & 0x7fffffffu, __float_as_uint(v.w) & 0x7fffffffu)));
      } else {
        for (long long j = i; j < n && j < i + 4; ++j) m = max(m, __float_as_uint(yb[j]) & 0x7fffffffu);
      }
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      m = max(max(part[0], part[1]), max(part[2], part[3]));
      atomicMax(amax_bits + b, m);
    }
    __syncthreads();  // part[] is reused by the next item
  }
}

template <class T>
hipError_t reorder_t(const Geom& g, const float* y, int b0, int nb, int btot, void* ws,
                     hipStream_t st) {
  const long long nqmk = (long long)g.Q * g.M * g.K;
  T* out = static_cast<T*>(ws);
  if constexpr (__is_same(T, uint8_t)) {
    hipError_t e = launch_item_absmax(g, y, b0, nb, const_cast<float*>(g.amax), st);
    if (e != hipSuccess) return e;
  }
  const bool aligned = (reinterpret_cast<uintptr_t>(y) & 15) == 0 &&
                       (reinterpret_cast<uintptr_t>(ws) & (4 * sizeof(T) - 1)) == 0;
  if (nb == 1 && btot == 1 && aligned && nqmk % 4 == 0) {
    const size_t n4 = (size_t)nqmk / 4;
    const size_t blocks = (n4 + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    hipLaunchKernelGGL(copy_convert_contig<T>, dim3((unsigned)blocks), dim3(256), 0, st, y, n4, out,
                       g.amax, b0);
  } else if (nb == 1 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    const size_t blocks = (size_t)std::min<long long>((nqmk / 4 + 255) / 256 + 1, 65536);
    hipLaunchKernelGGL(copy_convert<T>, dim3((unsigned)blocks), dim3(256), 0, st, y,
                       (size_t)nqmk, out, (size_t)btot, (size_t)b0, g.amax);
  } else {
    dim3 grid((unsigned)((nqmk + 63) / 64), (unsigned)((nb + 63) / 64));
    hipLaunchKernelGGL(transpose_convert<T>, grid, dim3(256), 0, st, y, nqmk, nb, b0, btot, out,
                       g.amax);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_item_absmax(const Geom& g, const float* y, int b0, int nb, float* amax,
                              hipStream_t st) {
  if (!amax) return hipErrorInvalidValue;
  unsigned* bits = reinterpret_cast<unsigned*>(amax) + b0;
  hipLaunchKernelGGL(zero_items, dim3((nb + 255) / 256), dim3(256), 0, st, bits, nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long n = (long long)g.Q * g.M * g.K;
  const unsigned bx = (unsigned)std::max<long long>(1, std::min<long long>((n / 4 + 255) / 256, 512));
  hipLaunchKernelGGL(item_absmax, dim3(bx, (unsigned)std::min(nb, 65535)), dim3(256), 0, st, y, n,
                     nb, bits);
  return hipGetLastError();
}

hipError_t launch_reorder(const Geom& g, int storage, const float* y, int b0, int nb, int btot,
                          void* ws, hipStream_t st) {
  switch (storage) {
    case DAS_STORE_F32: return reorder_t<float>(g, y, b0, nb, btot, ws, st);
    case DAS_STORE_F16: return reorder_t<_Float16>(g, y, b0, nb, btot, ws, st);
    case DAS_STORE_FP8_E4M3: return reorder_t<uint8_t>(g, y, b0, nb, btot, ws, st);
    default: return reorder_t<uint16_t>(g, y, b0, nb, btot, ws, st);
  }
}

}  // namespace dasmi
