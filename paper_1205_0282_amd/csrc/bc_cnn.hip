// Learned upsampler: a three-layer 3x3 convolutional network that turns a
// half-resolution, coarse-step render into a full-resolution image
// (no passage in the paper; the network is a stated reading):
//
//   a1 = relu(conv(x;  W1 32x4))   a2 = relu(conv(a1; W2 32x32))
//   y  = conv(a2; W3 16x32)        out = pixel_shuffle2(y) + bilinear2(x)
//
// Every convolution is an implicit GEMM on the matrix cores: rows are output
// pixels, columns output channels, and the reduction runs over (tap, input
// channel) in steps of 32 with v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32
// accumulation).  Operand B (weights) is pre-packed per (k-step, n-tile) in
// the lane order of the instruction, so one 16-byte load per lane feeds one
// MFMA.  Operand A is read from an LDS tile of the layer input (NHWC, BF16).
//
// Kernels: fused inference (all three layers of a 16x16 output tile with
// LDS-resident activations), per-layer training forward with the loss in the
// last layer's epilogue, backward-data (a forward convolution with flipped,
// channel-transposed weights and the ReLU mask in the epilogue),
// backward-weights (GEMM over the pixels of a tile, partial sums per tile,
// then a deterministic reduction), Adam, and the weight packer.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "bc_cnn.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// round to nearest, ties to even (one hardware conversion on gfx950)
__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// ------------------------------------------------------------------ A operand
// Lane (g = lane/16, r = lane%16) of an M-tile supplies row r (output pixel p)
// and reduction indices k0 .. k0+7 with k0 = 32 ks + 8 g; k = tap*CIN + c.
// `in` is an LDS tile, WIN pixels wide, SIN BF16 elements per pixel; the
// output pixel with input offset `pix` (its element index in the tile) reads
// input pixel pix + dy*WIN + dx for tap dy*3 + dx.  Tile shapes are template
// parameters, so that with the k-steps unrolled every tap offset is a
// constant of the LDS instruction.
template <int CIN, int WIN, int SIN>
__device__ __forceinline__ int tap_offset(int tap) {
  return tap < 9 ? ((tap / 3) * WIN + tap % 3) * SIN : -1;
}

// element offsets (from the output pixel's input position) of the lane's
// reduction indices at k-step ks: for CIN >= 8 one run of 8 channels of one
// tap, for CIN = 4 two taps of 4 channels; -1 for the zero padding past tap 8
template <int CIN, int WIN, int SIN>
__device__ __forceinline__ int2 lane_offsets(int g, int ks) {
  if (CIN >= 8) {
    // CIN = 32: tap = ks, channel 8 g; CIN = 16: tap = 2 ks + g/2, channel 8 (g%2)
    const int o = tap_offset<CIN, WIN, SIN>(ks * (32 / CIN) + (8 * g) / CIN);
    return make_int2(o < 0 ? -1 : o + (8 * g) % CIN, -1);
  }
  const int t0 = (ks * 32 + 8 * g) / 4;
  return make_int2(tap_offset<CIN, WIN, SIN>(t0), tap_offset<CIN, WIN, SIN>(t0 + 1));
}

template <int CIN>
__device__ __forceinline__ bf16x8 load_a(const uint16_t* in, int pix, int2 off) {
  if (CIN >= 8) {
    if (off.x < 0) return as_bf16x8(make_uint4(0, 0, 0, 0));
    return as_bf16x8(*reinterpret_cast<const uint4*>(in + pix + off.x));
  }
  const uint2 h0 = off.x >= 0 ? *reinterpret_cast<const uint2*>(in + pix + off.x) : make_uint2(0, 0);
  const uint2 h1 = off.y >= 0 ? *reinterpret_cast<const uint2*>(in + pix + off.y) : make_uint2(0, 0);
  return as_bf16x8(make_uint4(h0.x, h0.y, h1.x, h1.y));
}

// wave-uniform buffer resource over `bytes` bytes at `base` (scalar registers)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(const void* base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* ub = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)bytes, 0x00020000);
}

// One convolution layer over an LDS tile: M output pixels in raster order of
// an output tile WOUT wide; KS k-steps, NT n-tiles of packed weights `wf`
// (read through a buffer resource: one lane offset, the fragment offsets are
// constants).  A wave takes R of its M-tiles at a time, so that every weight
// fragment it loads feeds R matrix instructions (and R x NT accumulations are
// in flight).  epi(p0, v) receives the accumulated outputs (bias not added)
// of four consecutive pixels p0 .. p0+3 (those below M are valid): v[nt][i] is
// pixel p0 + i, channel 16 nt + (lane % 16); per-pixel work is done once for
// all the lane's channels.
template <int CIN, int KS, int NT, int R, int WIN, int SIN, int M, int WOUT, typename Epi>
__device__ __forceinline__ void conv_tile(const uint16_t* in, const uint4* __restrict__ wf, Epi epi) {
  // (every kernel here runs 256-thread workgroups: 4 waves; the wave index is
  // made explicitly uniform so that the per-tile guards below are scalar branches)
  constexpr int nwaves = 4;
  const int lane = threadIdx.x & 63, wave = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r = lane & 15;
  constexpr int n_mt = (M + 15) / 16;
  const __amdgpu_buffer_rsrc_t wr = wave_rsrc(wf, (uint32_t)(KS * NT * 64 * 16));
  // the lane's tap offsets do not depend on the pixel: computed once
  int2 off[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) off[ks] = lane_offsets<CIN, WIN, SIN>(g, ks);
  for (int base = wave; base < n_mt; base += nwaves * R) {
    f32x4 acc[R][NT];
    int pix[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int p = min((base + nwaves * j) * 16 + r, M - 1);
      pix[j] = ((p / WOUT) * WIN + p % WOUT) * SIN;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[j][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      bf16x8 a[R];
#pragma unroll
      for (int j = 0; j < R; ++j) a[j] = load_a<CIN>(in, pix[j], off[ks]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        const u4 w = __builtin_amdgcn_raw_buffer_load_b128(wr, lane * 16, (ks * NT + nt) * 1024, 0);
        const bf16x8 b = __builtin_bit_cast(bf16x8, w);
        // (every slot is computed: a slot past the last M-tile reads clamped
        // pixels and is not stored; a guard here would cost more than it saves)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[j][nt] = mfma(a[j], b, acc[j][nt]);
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int mt = base + nwaves * j;
      if (mt >= n_mt) break;
      epi(mt * 16 + 4 * g, acc[j]);
    }
  }
}

// fine-pixel value of the bilinear x2 upsampling of channel c of x (FP32,
// half-pixel centres, clamp to edge)
__device__ __forceinline__ float bilinear2(const float* __restrict__ x, int H, int W, int Y, int X, int c) {
  const float cy = ((float)Y + 0.5f) * 0.5f - 0.5f, cx = ((float)X + 0.5f) * 0.5f - 0.5f;
  const float fy0 = floorf(cy), fx0 = floorf(cx);
  const float fy = cy - fy0, fx = cx - fx0;
  const int y0 = min(max((int)fy0, 0), H - 1), y1 = min(max((int)fy0 + 1, 0), H - 1);
  const int x0 = min(max((int)fx0, 0), W - 1), x1 = min(max((int)fx0 + 1, 0), W - 1);
  const float v00 = x[((int64_t)y0 * W + x0) * 4 + c], v01 = x[((int64_t)y0 * W + x1) * 4 + c];
  const float v10 = x[((int64_t)y1 * W + x0) * 4 + c], v11 = x[((int64_t)y1 * W + x1) * 4 + c];
  const float top = v00 * (1.0f - fx) + v01 * fx;
  const float bot = v10 * (1.0f - fx) + v11 * fx;
  return top * (1.0f - fy) + bot * fy;
}

constexpr int PSTRIDE = 32;   // BF16 elements per pixel of a 32-channel LDS tile (64 B, 16-B aligned): the fused
                               // inference then takes 51 KB of LDS, so three workgroups fit a CU (45.8 us per
                               // 960x540 frame, against 52.2 us with 80-B pixels and two workgroups, despite
                               // more bank conflicts)

// ------------------------------------------------------------------ inference
// One 16x16 tile of coarse pixels per workgroup: input tile with a 3-pixel
// halo, both hidden activations in LDS, output 32x32 fine pixels.  The last
// layer's results go to an LDS output tile (in the first activation's space,
// free by then) and leave as whole fine pixels, with the bilinear skip read
// from an FP32 copy of the input (in the BF16 input tile's space, free after
// the first layer).
constexpr int XF = 18;   // FP32 input pixels per side for the bilinear skip of a tile
__global__ __launch_bounds__(256) void infer_kernel(CnnInferArgs a) {
  __shared__ __attribute__((aligned(16))) float xbuf[XF * XF * 4];   // BF16 22x22x4 input, then FP32 18x18x4
  __shared__ __attribute__((aligned(16))) uint16_t a1[20 * 20 * PSTRIDE];
  __shared__ __attribute__((aligned(16))) uint16_t a2[18 * 18 * PSTRIDE];
  static_assert(sizeof(uint16_t) * 22 * 22 * 4 <= sizeof(float) * XF * XF * 4, "input tile fits");
  static_assert(sizeof(uint16_t) * 20 * 20 * PSTRIDE >= sizeof(float) * 32 * 32 * 4, "output tile fits");
  uint16_t* xs = reinterpret_cast<uint16_t*>(xbuf);
  const int H = a.h, W = a.w;
  const int n = blockIdx.z;
  const int oy = blockIdx.y * 16, ox = blockIdx.x * 16;
  const float* __restrict__ x = a.x + (int64_t)n * H * W * 4;
  float* __restrict__ out = a.out + (int64_t)n * 4 * H * W * 4;
  const float* __restrict__ bias = a.params;
  for (int i = threadIdx.x; i < 22 * 22; i += blockDim.x) {
    const int gy = oy - 3 + i / 22, gx = ox - 3 + i % 22;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = reinterpret_cast<const float4*>(x)[(int64_t)gy * W + gx];
    xs[i * 4 + 0] = bf16_bits(v.x);
    xs[i * 4 + 1] = bf16_bits(v.y);
    xs[i * 4 + 2] = bf16_bits(v.z);
    xs[i * 4 + 3] = bf16_bits(v.w);
  }
  __syncthreads();
  const int r16 = threadIdx.x & 15;
  const float b1a = bias[CNN_OFF_B1 + r16], b1b = bias[CNN_OFF_B1 + 16 + r16];
  conv_tile<4, 2, 2, 4, 22, 4, 400, 20>(xs, a.wf1, [&](int p0, const f32x4* v) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + i;
      if (p >= 400) break;
      const int gy = oy - 2 + p / 20, gx = ox - 2 + p % 20;
      const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
      uint16_t* d = a1 + p * PSTRIDE + r16;
      d[0] = in ? bf16_bits(fmaxf(v[0][i] + b1a, 0.0f)) : (uint16_t)0;
      d[16] = in ? bf16_bits(fmaxf(v[1][i] + b1b, 0.0f)) : (uint16_t)0;
    }
  });
  __syncthreads();
  // FP32 input rows oy-1 .. oy+16 and columns ox-1 .. ox+16, clamped to the
  // image as the bilinear skip clamps them
  for (int i = threadIdx.x; i < XF * XF; i += blockDim.x) {
    const int gy = min(max(oy - 1 + i / XF, 0), H - 1), gx = min(max(ox - 1 + i % XF, 0), W - 1);
    reinterpret_cast<float4*>(xbuf)[i] = reinterpret_cast<const float4*>(x)[(int64_t)gy * W + gx];
  }
  const float b2a = bias[CNN_OFF_B2 + r16], b2b = bias[CNN_OFF_B2 + 16 + r16];
  conv_tile<32, 9, 2, 3, 20, PSTRIDE, 324, 18>(a1, a.wf2, [&](int p0, const f32x4* v) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + i;
      if (p >= 324) break;
      const int gy = oy - 1 + p / 18, gx = ox - 1 + p % 18;
      const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
      uint16_t* d = a2 + p * PSTRIDE + r16;
      d[0] = in ? bf16_bits(fmaxf(v[0][i] + b2a, 0.0f)) : (uint16_t)0;
      d[16] = in ? bf16_bits(fmaxf(v[1][i] + b2b, 0.0f)) : (uint16_t)0;
    }
  });
  __syncthreads();
  float* ot = reinterpret_cast<float*>(a1);   // [32][32] fine pixels x 4 channels
  // the lane's output channel 4c + 2dy + dx goes to fine pixel (2i + dy, 2j + dx), channel c
  const float b3v = bias[CNN_OFF_B3 + r16];
  const int c3 = r16 >> 2, dy3 = (r16 >> 1) & 1, dx3 = r16 & 1;
  conv_tile<32, 9, 1, 4, 18, PSTRIDE, 256, 16>(a2, a.wf3, [&](int p0, const f32x4* v) {
    // p0 .. p0+3 lie in one row of the 16-pixel-wide tile
    float* d = ot + ((2 * (p0 / 16) + dy3) * 32 + 2 * (p0 % 16) + dx3) * 4 + c3;
#pragma unroll
    for (int i = 0; i < 4; ++i) d[8 * i] = v[0][i] + b3v;
  });
  __syncthreads();
  // out = shuffled network output + bilinear x2 of x (half-pixel centres,
  // clamp to edge), whole fine pixels per thread
  for (int i = threadIdx.x; i < 32 * 32; i += blockDim.x) {
    const int fy = i / 32, fx = i % 32;
    const int Y = 2 * oy + fy, X = 2 * ox + fx;
    if (Y >= 2 * H || X >= 2 * W) continue;
    const float cy = ((float)Y + 0.5f) * 0.5f - 0.5f, cx = ((float)X + 0.5f) * 0.5f - 0.5f;
    const float fy0 = floorf(cy), fx0 = floorf(cx);
    const float ty = cy - fy0, tx = cx - fx0;
    const int y0 = min(max((int)fy0, 0), H - 1) - (oy - 1), y1 = min(max((int)fy0 + 1, 0), H - 1) - (oy - 1);
    const int x0 = min(max((int)fx0, 0), W - 1) - (ox - 1), x1 = min(max((int)fx0 + 1, 0), W - 1) - (ox - 1);
    const float4 v00 = reinterpret_cast<const float4*>(xbuf)[y0 * XF + x0];
    const float4 v01 = reinterpret_cast<const float4*>(xbuf)[y0 * XF + x1];
    const float4 v10 = reinterpret_cast<const float4*>(xbuf)[y1 * XF + x0];
    const float4 v11 = reinterpret_cast<const float4*>(xbuf)[y1 * XF + x1];
    const float4 z = reinterpret_cast<const float4*>(ot)[i];
    auto bl = [&](float a00, float a01, float a10, float a11) {
      const float top = a00 * (1.0f - tx) + a01 * tx;
      const float bot = a10 * (1.0f - tx) + a11 * tx;
      return top * (1.0f - ty) + bot * ty;
    };
    float4 o;
    o.x = z.x + bl(v00.x, v01.x, v10.x, v11.x);
    o.y = z.y + bl(v00.y, v01.y, v10.y, v11.y);
    o.z = z.z + bl(v00.z, v01.z, v10.z, v11.z);
    o.w = z.w + bl(v00.w, v01.w, v10.w, v11.w);
    reinterpret_cast<float4*>(out)[(int64_t)Y * 2 * W + X] = o;
  }
}

// ------------------------------------------------------------------ training forward / backward-data
// Stage an 18x18 input tile (output tile 16x16 plus a 1-pixel halo) of CIN
// channels into LDS: from the FP32 image (CIN = 4) or a BF16 NHWC tensor.
template <int CIN>
__device__ void stage_tile(uint16_t* t, int sin, const float* __restrict__ img, const uint16_t* __restrict__ act,
                           int H, int W, int oy, int ox) {
  for (int i = threadIdx.x; i < 18 * 18; i += blockDim.x) {
    const int gy = oy - 1 + i / 18, gx = ox - 1 + i % 18;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    if (CIN == 4) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (in) v = reinterpret_cast<const float4*>(img)[(int64_t)gy * W + gx];
      t[i * sin + 0] = bf16_bits(v.x);
      t[i * sin + 1] = bf16_bits(v.y);
      t[i * sin + 2] = bf16_bits(v.z);
      t[i * sin + 3] = bf16_bits(v.w);
    } else {
      const uint4* src = reinterpret_cast<const uint4*>(act + ((int64_t)gy * W + gx) * CIN);
      for (int q = 0; q < CIN / 8; ++q)
        *reinterpret_cast<uint4*>(t + i * sin + 8 * q) = in ? src[q] : make_uint4(0, 0, 0, 0);
    }
  }
}

// mode 0: a = bf16(relu(z + b)) stored NHWC (COUT channels)
// mode 1: g = bf16(z * [mask > 0]) stored NHWC (backward-data with ReLU mask)
// mode 2: last layer + loss: y = z + b, out = shuffle(y) + bilinear(x),
//         g_y = bf16(2 (out - target) / count), squared error summed per tile
template <int CIN, int COUT, int KS, int MODE>
__global__ __launch_bounds__(256) void layer_kernel(CnnLayerArgs a) {
  constexpr int SIN = CIN == 4 ? 4 : PSTRIDE;
  __shared__ __attribute__((aligned(16))) uint16_t t[18 * 18 * SIN];
  __shared__ float red[256];
  const int H = a.h, W = a.w;
  const int n = blockIdx.z;
  const int oy = blockIdx.y * 16, ox = blockIdx.x * 16;
  const int64_t plane = (int64_t)H * W;
  stage_tile<CIN>(t, SIN, a.img ? a.img + n * plane * 4 : nullptr, a.in ? a.in + n * plane * CIN : nullptr, H, W, oy, ox);
  __syncthreads();
  float sq = 0.0f;
  constexpr int NT = COUT / 16;
  const int r16 = threadIdx.x & 15;
  float bv[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) bv[nt] = MODE == 1 ? 0.0f : a.bias[16 * nt + r16];
  conv_tile<CIN, KS, NT, 4, 18, SIN, 256, 16>(t, a.wf, [&](int p0, const f32x4* v) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = p0 + i;
      const int gy = oy + p / 16, gx = ox + p % 16;
      if (gy >= H || gx >= W) continue;
      const int64_t pix = n * plane + (int64_t)gy * W + gx;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = 16 * nt + r16;
        const float z = v[nt][i];
        if (MODE == 0) {
          a.out[pix * COUT + c] = bf16_bits(fmaxf(z + bv[nt], 0.0f));
        } else if (MODE == 1) {
          a.out[pix * COUT + c] = (a.mask[pix * COUT + c] & 0x7fffu) != 0 ? bf16_bits(z) : (uint16_t)0;
        } else {
          const float* xi = a.img + n * plane * 4;
          const int ch = c >> 2, dy = (c >> 1) & 1, dx = c & 1;
          const int Y = 2 * gy + dy, X = 2 * gx + dx;
          const int64_t fi = ((int64_t)n * 4 * plane + (int64_t)Y * 2 * W + X) * 4 + ch;
          const float o = (z + bv[nt]) + bilinear2(xi, H, W, Y, X, ch);
          const float d = o - a.target[fi];
          sq += d * d;
          a.out[pix * COUT + c] = bf16_bits(d * a.grad_scale);
        }
      }
    }
  });
  if (MODE == 2) {
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      a.loss_part[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
  }
}

// ------------------------------------------------------------------ backward-weights
// Per 16x16 tile: dW[o][c][tap] += sum_p g[p][o] x[p + tap][c] as a GEMM with
// rows o (COUT), columns n = tap*CIN + c, reduction over the tile's 256 pixels;
// db[o] += sum_p g[p][o].  Partial sums per tile go to `part`.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void wgrad_kernel(CnnWgradArgs a) {
  constexpr int SIN = CIN == 4 ? 4 : PSTRIDE;
  constexpr int NCOL = 9 * CIN;
  constexpr int NTN = (NCOL + 15) / 16;
  __shared__ __attribute__((aligned(16))) uint16_t xt[18 * 18 * SIN];
  __shared__ __attribute__((aligned(16))) uint16_t gt[256 * COUT];
  const int H = a.h, W = a.w;
  const int n = blockIdx.z;
  const int oy = blockIdx.y * 16, ox = blockIdx.x * 16;
  const int64_t plane = (int64_t)H * W;
  const int64_t tile = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  stage_tile<CIN>(xt, SIN, a.img ? a.img + n * plane * 4 : nullptr, a.x ? a.x + n * plane * CIN : nullptr, H, W, oy, ox);
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    const int gy = oy + i / 16, gx = ox + i % 16;
    const bool in = gy < H && gx < W;
    const uint4* src = reinterpret_cast<const uint4*>(a.g + (n * plane + (int64_t)gy * W + gx) * COUT);
    for (int q = 0; q < COUT / 8; ++q)
      *reinterpret_cast<uint4*>(gt + i * COUT + 8 * q) = in ? src[q] : make_uint4(0, 0, 0, 0);
  }
  __syncthreads();
  float* part = a.part + tile * (int64_t)(COUT * NCOL + COUT);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  for (int job = wave; job < (COUT / 16) * NTN; job += nwaves) {
    const int mt = job / NTN, nt = job % NTN;
    const int o = mt * 16 + r;
    const int col = nt * 16 + r;
    const bool cval = col < NCOL;
    const int tap = cval ? col / CIN : 0, c = cval ? col % CIN : 0;
    const int dy = tap / 3, dx = tap % 3;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < 8; ++ks) {
      uint16_t av[8], bv[8];
      for (int i = 0; i < 8; ++i) {
        const int p = ks * 32 + 8 * g + i;
        av[i] = gt[p * COUT + o];
        bv[i] = cval ? xt[((p / 16 + dy) * 18 + (p % 16) + dx) * SIN + c] : (uint16_t)0;
      }
      const uint4 ua = make_uint4(av[0] | (uint32_t)av[1] << 16, av[2] | (uint32_t)av[3] << 16,
                                  av[4] | (uint32_t)av[5] << 16, av[6] | (uint32_t)av[7] << 16);
      const uint4 ub = make_uint4(bv[0] | (uint32_t)bv[1] << 16, bv[2] | (uint32_t)bv[3] << 16,
                                  bv[4] | (uint32_t)bv[5] << 16, bv[6] | (uint32_t)bv[7] << 16);
      acc = mfma(as_bf16x8(ua), as_bf16x8(ub), acc);
    }
    if (cval)
      for (int i = 0; i < 4; ++i) {
        const int oo = mt * 16 + 4 * g + i;
        part[oo * NCOL + c * 9 + tap] = acc[i];   // layout W[o][c][dy][dx]
      }
  }
  if ((int)threadIdx.x < COUT) {
    float s = 0.0f;
    for (int p = 0; p < 256; ++p) s += bf16_float(gt[p * COUT + threadIdx.x]);
    part[COUT * NCOL + threadIdx.x] = s;
  }
}

// sum of the per-tile partials into the flat gradient (fixed order: deterministic)
__global__ void reduce_kernel(const float* __restrict__ part, int64_t n_tiles, int width, float* __restrict__ grad_w,
                              float* __restrict__ grad_b, int n_w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= width) return;
  float s = 0.0f;
  for (int64_t t = 0; t < n_tiles; ++t) s += part[t * width + j];
  if (j < n_w) grad_w[j] = s;
  else grad_b[j - n_w] = s;
}

// ------------------------------------------------------------------ Adam and packing
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// B fragments: element i of lane l of (ks, nt) is B[k][n] with
// k = 32 ks + 8 (l / 16) + i, n = 16 nt + l % 16.  Forward layers:
// B[tap*CIN + c][o] = W[o][c][tap]; backward-data (a convolution of the output
// gradient): B[tap*COUT + o][c] = W[o][c][8 - tap].
__global__ void pack_kernel(const float* __restrict__ w, CnnPackTable tab) {
  const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
  int rem = gidx;
  for (int e = 0; e < tab.n; ++e) {
    const CnnPackEntry& p = tab.e[e];
    const int count = p.ks * p.nt * 64 * 8;
    if (rem < count) {
      const int i = rem & 7, lane = (rem >> 3) & 63, frag = rem >> 9;
      const int ks = frag / p.nt, nt = frag % p.nt;
      const int k = 32 * ks + 8 * (lane >> 4) + i, ncol = 16 * nt + (lane & 15);
      float val = 0.0f;
      if (!p.transposed) {
        // forward: k = tap*cin + c, ncol = o
        if (k < 9 * p.cin) {
          const int tap = k / p.cin, c = k % p.cin;
          val = w[p.w_off + (ncol * p.cin + c) * 9 + tap];
        }
      } else {
        // backward-data: k = tap*cout + o, ncol = c
        if (k < 9 * p.cout) {
          const int tap = k / p.cout, o = k % p.cout;
          val = w[p.w_off + (o * p.cin + ncol) * 9 + (8 - tap)];
        }
      }
      p.dst[rem] = bf16_bits(val);
      return;
    }
    rem -= count;
  }
}

}  // namespace

hipError_t cnn_launch_infer(const CnnInferArgs& a, int n, hipStream_t st) {
  dim3 grid((a.w + 15) / 16, (a.h + 15) / 16, n);
  infer_kernel<<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t cnn_launch_layer(int layer, int mode, const CnnLayerArgs& a, int n, hipStream_t st) {
  dim3 grid((a.w + 15) / 16, (a.h + 15) / 16, n);
  if (layer == 1 && mode == 0) layer_kernel<4, 32, 2, 0><<<grid, 256, 0, st>>>(a);
  else if (layer == 2 && mode == 0) layer_kernel<32, 32, 9, 0><<<grid, 256, 0, st>>>(a);
  else if (layer == 3 && mode == 2) layer_kernel<32, 16, 9, 2><<<grid, 256, 0, st>>>(a);
  // backward-data of layer 3: input g_y (16 ch) -> g_a2 (32 ch) masked by a2
  else if (layer == 3 && mode == 1) layer_kernel<16, 32, 5, 1><<<grid, 256, 0, st>>>(a);
  // backward-data of layer 2: input g_z2 (32 ch) -> g_a1 (32 ch) masked by a1
  else if (layer == 2 && mode == 1) layer_kernel<32, 32, 9, 1><<<grid, 256, 0, st>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t cnn_launch_wgrad(int layer, const CnnWgradArgs& a, int n, hipStream_t st) {
  dim3 grid((a.w + 15) / 16, (a.h + 15) / 16, n);
  if (layer == 1) wgrad_kernel<4, 32><<<grid, 256, 0, st>>>(a);
  else if (layer == 2) wgrad_kernel<32, 32><<<grid, 256, 0, st>>>(a);
  else if (layer == 3) wgrad_kernel<32, 16><<<grid, 256, 0, st>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t cnn_launch_reduce(const float* part, int64_t n_tiles, int width, float* grad_w, float* grad_b, int n_w,
                             hipStream_t st) {
  reduce_kernel<<<(width + 255) / 256, 256, 0, st>>>(part, n_tiles, width, grad_w, grad_b, n_w);
  return hipGetLastError();
}

hipError_t cnn_launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, int64_t step,
                           hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, (double)step)), c2 = (float)(1.0 - pow(b2, (double)step));
  adam_kernel<<<(n + 255) / 256, 256, 0, st>>>(w, m, v, g, n, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t cnn_launch_pack(const float* w, const CnnPackTable& tab, hipStream_t st) {
  int total = 0;
  for (int e = 0; e < tab.n; ++e) total += tab.e[e].ks * tab.e[e].nt * 64 * 8;
  pack_kernel<<<(total + 255) / 256, 256, 0, st>>>(w, tab);
  return hipGetLastError();
}
