// Building blocks of the matrix-core (MFMA) forms (k_mfma.hip, k_mfma_wg.hip):
// operand types and conversions, the A-fragment placement of a voxel's two
// interpolation weights, the receive-cone test of a voxel box, and DPP row
// reductions.  gfx950 only.
#pragma once
#include "das_device.h"
#include "fp8.h"

namespace dasmi {
namespace mfma {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf168 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int CH = 8;  // samples per chunk

__device__ inline uint16_t f16_bits(float v) {
  const _Float16 h = (_Float16)v;
  return __builtin_bit_cast(uint16_t, h);
}
// float -> bf16 bits, round to nearest even, NaN kept quiet.
__device__ inline uint16_t bf16_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(float v) { return __uint_as_float((uint32_t)bf16_bits(v) << 16); }

// Put the packed pair P = (w1, w2) at 16-bit slots (d, d+1) of an 8-slot
// fragment; slots outside [0, 8) are dropped.
__device__ inline u32x4 place_pair(uint32_t P, int d) {
  const uint64_t x = P;
  const int d1 = d - 4;
  const uint64_t lo = ((unsigned)d <= 3u) ? (x << ((16 * d) & 63)) : (d == -1 ? (x >> 16) : 0ull);
  const uint64_t hi = ((unsigned)d1 <= 3u) ? (x << ((16 * d1) & 63)) : (d1 == -1 ? (x >> 16) : 0ull);
  return u32x4{(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
}

// The same for 8-bit slots: the two codes (w1, w2) of P's low 16 bits at
// byte slots (d, d+1) of an 8-byte fragment.
__device__ inline u32x2 place_pair8(uint32_t P, int d) {
  const uint64_t x = P & 0xffffu;
  const uint64_t v = ((unsigned)d <= 7u) ? (x << ((8 * d) & 63)) : (d == -1 ? (x >> 8) : 0ull);
  return u32x2{(uint32_t)v, (uint32_t)(v >> 32)};
}

// Interpolation weights as A operands.  pack2 writes the operand bits of the
// pair (w1, w2) into hi and, for split types, the operand bits of the
// remainder (w - value(hi)) into lo: two MFMAs with the same B fragment then
// carry the weights with a relative error of about the operand's precision
// squared.  Weights are multiplied by kScale before rounding (the output is
// divided by it).
template <class T> struct Mma;
template <> struct Mma<_Float16> {
  static constexpr bool kSplit = false;
  static constexpr float kScale = 1.f;
  using Frag = u32x4;
  __device__ static f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, a),
                                                   __builtin_bit_cast(half8, b), c, 0, 0, 0);
  }
  __device__ static uint32_t pack(float a, float b) {
    return (uint32_t)f16_bits(a) | ((uint32_t)f16_bits(b) << 16);
  }
  __device__ static void pack2(float a, float b, uint32_t& hi, uint32_t& lo) {
    hi = pack(a, b);
    lo = 0u;
  }
  __device__ static Frag place(uint32_t P, int d) { return place_pair(P, d); }
};
template <> struct Mma<uint16_t> {  // bf16 bit patterns
  static constexpr bool kSplit = true;
  static constexpr float kScale = 1.f;
  using Frag = u32x4;
  __device__ static f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf168, a),
                                                    __builtin_bit_cast(bf168, b), c, 0, 0, 0);
  }
  __device__ static uint32_t pack(float a, float b) {
    return (uint32_t)bf16_bits(a) | ((uint32_t)bf16_bits(b) << 16);
  }
  __device__ static void pack2(float a, float b, uint32_t& hi, uint32_t& lo) {
    hi = pack(a, b);
    lo = pack(a - bf16_value(a), b - bf16_value(b));
  }
  __device__ static Frag place(uint32_t P, int d) { return place_pair(P, d); }
};
// FP8 (E4M3) operands on both sides: v_mfma_f32_16x16x32_fp8_fp8 contracts the
// stored sample codes directly (no decode); the weights, scaled by 2^7 (at
// most 128, below the largest E4M3 value 448, and clear of the subnormal
// range for weights down to ~1e-4), are split into two E4M3 parts.
struct Fp8Tag {};
template <> struct Mma<Fp8Tag> {
  static constexpr bool kSplit = true;
  static constexpr float kScale = 128.f;
  using Frag = u32x2;
  __device__ static f32x4 mma(u32x2 a, u32x2 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                       __builtin_bit_cast(long, b), c, 0, 0, 0);
  }
  __device__ static void pack2(float a, float b, uint32_t& hi, uint32_t& lo) {
    const float sa = a * kScale, sb = b * kScale;
    hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(sa, sb, 0, false) & 0xffffu;
    const float ra = sa - __builtin_amdgcn_cvt_f32_fp8((int)hi, 0);
    const float rb = sb - __builtin_amdgcn_cvt_f32_fp8((int)hi, 1);
    lo = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(ra, rb, 0, false) & 0xffffu;
  }
  __device__ static Frag place(uint32_t P, int d) { return place_pair8(P, d); }
};

// Workspace element type S -> MFMA operand type T and B-fragment load (8
// samples of one batch item).  f16 and bf16 are stored as operands; FP8 E4M3
// codes (8 bytes) are decoded to f16 in registers (exact), so the weights
// stay f16 and only the bytes moved shrink.
template <class S> struct Operand {
  using T = S;
  using Raw = u32x4;
  using Frag = u32x4;
  __device__ static Raw load(const S* p) { return *reinterpret_cast<const u32x4*>(p); }
  __device__ static u32x4 decode(Raw r) { return r; }
};
template <> struct Operand<uint8_t> {
  using T = _Float16;
  using Raw = u32x2;
  using Frag = u32x4;
  __device__ static Raw load(const uint8_t* p) { return *reinterpret_cast<const u32x2*>(p); }
  __device__ static u32x4 decode(Raw r) {
    uint32_t a, b, c, d;
    e4m3x4_to_f16x4(r.x, a, b);
    e4m3x4_to_f16x4(r.y, c, d);
    return u32x4{a, b, c, d};
  }
};


// FP8 samples used as FP8 MFMA operands (8 codes, one 8-byte load, no decode).
struct OperandFp8Raw {
  using T = Fp8Tag;
  using Raw = u32x2;
  using Frag = u32x2;
  __device__ static Raw load(const uint8_t* p) { return *reinterpret_cast<const u32x2*>(p); }
  __device__ static u32x2 decode(Raw r) { return r; }
};

// Can any point of the sphere (centre p0, radius R) lie in the receive cone of
// the element (e = p0 - r_m, axis n, half-angle with cos cth, sin sth)?
// Conservative and trig-free: cos(phi) > cos(theta + beta).
__device__ inline bool sphere_in_cone(float ex, float ey, float ez, float nx, float ny, float nz,
                                      float R, float cth, float sth) {
  const float D2 = ex * ex + ey * ey + ez * ez;
  if (D2 <= R * R * 1.0001f) return true;
  const float invD = __builtin_amdgcn_rsqf(D2);
  const float cphi = (ex * nx + ey * ny + ez * nz) * invD;
  const float sb = R * invD;
  const float cb = __builtin_amdgcn_sqrtf(fmaxf(0.f, 1.f - sb * sb));
  return cphi > cth * cb - sth * sb - 1e-4f;
}

// Min / max over the 16 lanes of a DPP row (rotations by 1, 2, 4, 8); every
// lane of the row ends with the result.
__device__ inline int row_min(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x121, 0xf, 0xf, true));
  v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x122, 0xf, 0xf, true));
  v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, true));
  v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, true));
  return v;
}
__device__ inline int row_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x121, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x122, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, true));
  return v;
}

}  // namespace mfma
}  // namespace dasmi
