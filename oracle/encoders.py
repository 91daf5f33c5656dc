"""Storage encoders for the cube (TEST INFRASTRUCTURE ONLY -- see oracle/__init__).

The paper keeps FP32 voxels (Table 1 sizes are 4 bytes per voxel).  The FP16
and FP8 storage forms have no passage in the paper; they are written here from
the format definitions themselves:

* IEEE 754 binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits,
  subnormal quantum 2^-24, round to nearest, ties to even; overflow to inf.
* OCP 8-bit floating point, E4M3 ("fn" variant): 1 sign, 4 exponent bits
  (bias 7), 3 mantissa bits, no infinities, S.1111.111 is NaN, largest finite
  magnitude 448, subnormal quantum 2^-9.  Encoding rounds to nearest even and
  saturates to +-448.

Per-brick affine quantisation for FP8 (a stated reading): over all values a
brick stores (core and ghost voxels) o = fp32((min+max)/2) and
s = fp32((max-min)/896); if max == min then s = 1.  Encoding is
x = fp32(fp32(v - o) * fp32(1/s)) followed by RNE-saturating e4m3; decoding is
q*s + o (here in FP64).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


# ------------------------------------------------------------------- binary16
def f16_bits(x) -> np.ndarray:
    """Round float32 values to IEEE binary16; returns the uint16 bit patterns."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    out = np.zeros(x.shape, dtype=np.uint16)
    sign = np.signbit(x)
    a = np.abs(x)
    nan = np.isnan(x)
    fin = ~nan & ~np.isinf(x)
    # quantum of the binade containing a (subnormal quantum below 2^-14)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -14.0)
    # log2 may be off by one at binade edges: correct so that 2^e <= a < 2^(e+1)
    e = np.where((a >= 2.0 ** (e + 1)) & (a > 0), e + 1, e)
    e = np.where((a < 2.0 ** e) & (a >= 2.0 ** -14), e - 1, e)
    q = 2.0 ** (e - 10)
    r = np.rint(a / q)                         # ties to even
    v = r * q                                  # exact rounded magnitude
    inf = np.isinf(x) | (fin & (v >= 65536.0))
    # encode v into bits
    bits = np.zeros(x.shape, dtype=np.int64)
    a = np.where(fin, a, 0.0)
    v = np.where(fin, v, 0.0)
    sub = fin & ~inf & (v < 2.0 ** -14)
    bits[sub] = (v[sub] / 2.0 ** -24).astype(np.int64)
    nor = fin & ~inf & ~sub
    if np.any(nor):
        vn = v[nor]
        en = np.floor(np.log2(vn))
        en = np.where(vn >= 2.0 ** (en + 1), en + 1, en)
        en = np.where(vn < 2.0 ** en, en - 1, en)
        frac = (vn / 2.0 ** en - 1.0) * 1024.0
        bits[nor] = ((en + 15).astype(np.int64) << 10) | np.rint(frac).astype(np.int64)
    bits[inf] = 0x7C00
    bits[nan] = 0x7E00
    bits = bits | (sign.astype(np.int64) << 15)
    out[...] = bits.astype(np.uint16)
    return out


def f16_value(bits) -> np.ndarray:
    """Exact value of binary16 bit patterns (FP64)."""
    b = np.asarray(bits, dtype=np.int64)
    s = np.where((b >> 15) & 1, -1.0, 1.0)
    e = (b >> 10) & 31
    m = (b & 1023).astype(np.float64)
    val = np.where(e == 0, m * 2.0 ** -24, (1.0 + m / 1024.0) * 2.0 ** (e.astype(np.float64) - 15))
    val = np.where(e == 31, np.where(m == 0, np.inf, np.nan), val)
    return s * val


# ---------------------------------------------------------------------- e4m3
def e4m3_value(code) -> np.ndarray:
    """Exact value of OCP E4M3 codes (FP64); NaN for S.1111.111."""
    c = np.asarray(code, dtype=np.int64)
    s = np.where((c >> 7) & 1, -1.0, 1.0)
    e = (c >> 3) & 15
    m = (c & 7).astype(np.float64)
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * 2.0 ** (e.astype(np.float64) - 7))
    val = np.where((e == 15) & ((c & 7) == 7), np.nan, val)
    return s * val


def _e4m3_table():
    mags = e4m3_value(np.arange(0, 127))         # codes 0x00 .. 0x7E, ascending
    return mags


_E4M3_POS = _e4m3_table()


def e4m3_encode(x) -> np.ndarray:
    """Float32 values to E4M3 codes: round to nearest even on the E4M3 grid,
    saturate to +-448, NaN -> 0x7F (sign kept)."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    sign = np.signbit(x)
    a = np.abs(x)
    nan = np.isnan(x)
    a = np.where(nan, 0.0, np.minimum(a, E4M3_MAX))   # saturate (incl. inf)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.where((a >= 2.0 ** (e + 1)) & (a > 0), e + 1, e)
    e = np.where((a < 2.0 ** e) & (a > 0), e - 1, e)
    e = np.maximum(e, -6.0)                      # subnormal quantum 2^-9 below 2^-6
    q = 2.0 ** (e - 3)
    v = np.rint(a / q) * q                       # ties to even (grid spacing q)
    v = np.minimum(v, E4M3_MAX)                  # saturate
    code = np.searchsorted(_E4M3_POS, v)         # exact match on the grid
    assert np.all(_E4M3_POS[np.clip(code, 0, 126)] == v), "value not on the E4M3 grid"
    code = np.where(nan, 0x7F, code)
    return (code | (sign.astype(np.int64) << 7)).astype(np.uint8)


# --------------------------------------------------------- per-brick quantiser
def brick_scale_offset(vmin: float, vmax: float):
    """(s, o) as float32 for a brick whose stored values span [vmin, vmax]."""
    mn, mx = np.float32(vmin), np.float32(vmax)
    if mx == mn:
        return np.float32(1.0), mn
    o = np.float32(np.float32(mn + mx) / np.float32(2.0))
    s = np.float32(np.float32(mx - mn) / np.float32(896.0))
    return s, o


def fp8_encode_brick(values, s, o) -> np.ndarray:
    v = np.asarray(values, dtype=np.float32)
    inv = np.float32(np.float32(1.0) / np.float32(s))
    x = (v - np.float32(o)).astype(np.float32) * inv
    return e4m3_encode(x.astype(np.float32))


def fp8_decode_brick(codes, s, o) -> np.ndarray:
    return e4m3_value(codes) * float(s) + float(o)
