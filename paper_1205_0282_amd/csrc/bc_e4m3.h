// OCP FP8 E4M3 (no infinities, 0x7f/0xff are NaN, largest finite 448) as the
// brick pool's 8-bit storage form: round-to-nearest-even encode saturating at
// +-448, and a branch-free decode.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

__device__ __forceinline__ uint8_t bc_e4m3_encode(float x) {
  const uint32_t bits = __float_as_uint(x);
  const uint32_t sign = (bits >> 31) << 7;
  if (x != x) return (uint8_t)(sign | 0x7f);
  float a = fminf(fabsf(x), 448.0f);
  uint32_t code;
  if (a < 0.015625f) {                               // below 2^-6: quantum 2^-9
    code = (uint32_t)rintf(a * 512.0f);              // 0..8 (8 is the smallest normal)
  } else {
    int e = (int)((__float_as_uint(a) >> 23) & 255) - 127;   // 2^e <= a < 2^(e+1), e in [-6, 8]
    float r = rintf(ldexpf(a, 3 - e));               // in [8, 16]
    uint32_t m = (uint32_t)r;
    if (m == 16) { m = 8; e += 1; }
    code = ((uint32_t)(e + 7) << 3) | (m - 8);
  }
  return (uint8_t)(sign | code);
}

// The code's exponent and mantissa bits placed at the top of an FP32 mantissa
// form a number (normal or subnormal) that is 2^-120 times the code's value,
// so one exact power-of-two product decodes normal and subnormal codes alike.
__device__ __forceinline__ float bc_e4m3_decode(uint32_t c) {
  const float mag = __uint_as_float((c & 0x7fu) << 20) * 1.329227995784916e+36f;   // 2^120
  return __uint_as_float(__float_as_uint(mag) | ((c & 0x80u) << 24));
}
