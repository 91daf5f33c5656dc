// Double-float ("df") arithmetic on FP32 pairs (hi + lo, |lo| <= ulp(hi)/2).
// Used once per ray and per brick / sample chunk so that sample positions keep
// about 44 bits of precision while every per-sample operation stays FP32.
// Error-free transformations: Knuth's two-sum, Dekker's fast two-sum and the
// FMA-based exact product.  Contraction is switched off so that the compiler
// cannot fuse the additions these transformations rely on.
#pragma once
#include <hip/hip_runtime.h>

struct df { float hi, lo; };

__device__ __forceinline__ df df_make(float hi, float lo) { df r; r.hi = hi; r.lo = lo; return r; }
__device__ __forceinline__ df df_from(float a) { return df_make(a, 0.0f); }

__device__ __forceinline__ df two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return df_make(s, e);
}

__device__ __forceinline__ df fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float e = b - (s - a);
  return df_make(s, e);
}

__device__ __forceinline__ df two_prod(float a, float b) {
#pragma clang fp contract(off)
  float p = a * b;
  float e = __builtin_fmaf(a, b, -p);
  return df_make(p, e);
}

__device__ __forceinline__ df df_add(df a, df b) {
#pragma clang fp contract(off)
  df s = two_sum(a.hi, b.hi);
  df t = two_sum(a.lo, b.lo);
  s.lo = s.lo + t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo = s.lo + t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ df df_neg(df a) { return df_make(-a.hi, -a.lo); }
__device__ __forceinline__ df df_sub(df a, df b) { return df_add(a, df_neg(b)); }

__device__ __forceinline__ df df_mul(df a, df b) {
#pragma clang fp contract(off)
  df p = two_prod(a.hi, b.hi);
  float c = __builtin_fmaf(a.hi, b.lo, a.lo * b.hi);
  p.lo = p.lo + c;
  return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ df df_mul_f(df a, float b) {
#pragma clang fp contract(off)
  df p = two_prod(a.hi, b);
  p.lo = __builtin_fmaf(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

// a + b for a float b: the leading parts summed exactly, the trailing part
// added to the error once
__device__ __forceinline__ df df_add_f(df a, float b) {
#pragma clang fp contract(off)
  df s = two_sum(a.hi, b);
  s.lo = s.lo + a.lo;
  return fast_two_sum(s.hi, s.lo);
}

// a / b: quotient digits from the hardware reciprocal of b.hi (about 1 ulp),
// each taken against the exact remainder, so that the approximate reciprocal
// costs no accuracy; b.hi is a normal number at the call sites (ray
// directions and lengths of order one)
__device__ __forceinline__ df df_div(df a, df b) {
#pragma clang fp contract(off)
  const float rb = __builtin_amdgcn_rcpf(b.hi);
  float q1 = a.hi * rb;
  df r = df_sub(a, df_mul_f(b, q1));
  float q2 = r.hi * rb;
  r = df_sub(r, df_mul_f(b, q2));
  float q3 = r.hi * rb;
  df q = fast_two_sum(q1, q2);
  return df_add_f(q, q3);
}

__device__ __forceinline__ df df_sqrt(df a) {
#pragma clang fp contract(off)
  if (a.hi <= 0.0f) return df_from(0.0f);
  float x = __builtin_amdgcn_sqrtf(a.hi);   // about 1 ulp; the correction below refines it
  df x2 = two_prod(x, x);
  df r = df_sub(a, x2);
  float c = r.hi * (0.5f * __builtin_amdgcn_rcpf(x));
  return fast_two_sum(x, c);
}

// exact comparisons of normalised pairs
__device__ __forceinline__ bool df_lt(df a, df b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ bool df_ge(df a, df b) { return !df_lt(a, b); }
__device__ __forceinline__ df df_min(df a, df b) { return df_lt(a, b) ? a : b; }
__device__ __forceinline__ df df_max(df a, df b) { return df_lt(a, b) ? b : a; }

__device__ __forceinline__ float df_to_f(df a) { return a.hi + a.lo; }
