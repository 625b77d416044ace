// FP8 workspace storage: OCP E4M3 samples with one power-of-two scale per
// batch item.  Storage below 16 bits is the paper's first future direction
// (Sec. 5); the format is the OCP 8-bit floating-point "E4M3" (1 sign bit, 4
// exponent bits with bias 7, 3 fraction bits, no infinities, S.1111.111 =
// NaN, largest finite magnitude 448).
//
// An item whose largest magnitude is A = f 2^x (f in [0.5, 1)) is stored as
// y 2^e with e = 8 - x, which puts its samples in [-256, 256): well inside
// the range (no saturation) and 2^16 above the smallest subnormal.  The
// forward multiplies the item's output by 2^-e (exact).  The workspace keeps
// A per item (a table after the samples), and every kernel derives e from it
// with the same function.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dasmi {

// Scale exponent of an item of largest magnitude amax; 0 for amax = 0 or a
// non-finite amax (NaN or inf samples).
__device__ inline int fp8_item_exponent(float amax) {
  if (!(amax > 0.f) || !(amax <= 3.402823466e38f)) return 0;
  int x;
  (void)frexpf(amax, &x);
  return 8 - x;
}

// v -> E4M3 code: nearest value, ties to the even code; finite magnitudes
// from 448 up saturate to 448; NaN and +-inf give NaN (sign kept).
__device__ inline uint32_t e4m3_bits(float v) {
  const uint32_t s = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = fabsf(v);
  if (!(a <= 3.402823466e38f)) return s | 0x7fu;
  if (a >= 448.f) return s | 0x7eu;
  // subnormal range: steps of 2^-9; rounding up to 8 steps gives 2^-6, code 0x08
  if (a < 0.015625f) return s | (uint32_t)rintf(a * 512.f);
  const uint32_t u = __float_as_uint(a);
  const uint32_t e = (u >> 23) - 120u;  // E4M3 biased exponent, 1 .. 15
  const uint32_t mant = u & 0x7fffffu;
  const uint32_t r = mant >> 20, rem = mant & 0xfffffu;
  const uint32_t up = (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ? 1u : 0u;
  return s | ((e << 3) + r + up);  // a carry out of the fraction steps the exponent
}

// E4M3 code (low byte) -> f32, exact.
__device__ inline float e4m3_to_f32(uint32_t code) {
  return __builtin_amdgcn_cvt_scalef32_f32_fp8(code, 1.0f, 0);
}

// Four E4M3 codes of a dword -> two dwords of two f16 each (exact: every
// E4M3 value is an f16 value).
__device__ inline void e4m3x4_to_f16x4(uint32_t w, uint32_t& lo, uint32_t& hi) {
  lo = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w, 1.0f, false));
  hi = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w, 1.0f, true));
}

}  // namespace dasmi
