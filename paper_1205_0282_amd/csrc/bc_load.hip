// Load-time kernels: per-brick minimum/maximum of the stored values (the
// paper's min/max task after the data reaches GPU memory, Section 2.3.1), the
// FP8 scale/offset, the largest decoded value, and the encode + layout of
// ghosted bricks into 4x4x4 micro-blocks (micro-blocks row-major inside the
// brick; a micro-block is 16 rows of 5 elements, x fastest, the fifth
// repeating the first voxel of the next micro-block along x).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include "bc_types.h"
#include "bc_kernels.h"
#include "bc_e4m3.h"

namespace {

__device__ __forceinline__ uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

template <typename T> __device__ __forceinline__ float to_f32(T v);
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }

struct SrcView {
  const void* ptr;
  int64_t sx, sy, sz;   // strides (elements)
  int32_t ox, oy, oz;   // global voxel coordinates of element [0][0][0]
  int32_t nx, ny, nz;   // global cube dims (for clamping)
};

template <typename T>
__device__ __forceinline__ float src_at(const SrcView& s, int gx, int gy, int gz) {
  gx = min(max(gx, 0), s.nx - 1);
  gy = min(max(gy, 0), s.ny - 1);
  gz = min(max(gz, 0), s.nz - 1);
  const T* p = static_cast<const T*>(s.ptr);
  return to_f32<T>(p[(int64_t)(gx - s.ox) * s.sx + (int64_t)(gy - s.oy) * s.sy + (int64_t)(gz - s.oz) * s.sz]);
}

// min/max over each brick's ghosted region [lo-1, hi+1) (clamped to the
// cube): brick first + blockIdx.y; every wave takes whole rows along x (32-bit
// index arithmetic, coalesced loads) and folds them into the brick's pair
template <typename T>
__global__ __launch_bounds__(256) void minmax_kernel(SrcView s, const BcBrick* __restrict__ bricks, int first,
                                                     BcCounters* ctr) {
  const int b = first + (int)blockIdx.y;
  const BcBrick& br = bricks[b];
  const int ex = br.hi[0] - br.lo[0] + 2, ey = br.hi[1] - br.lo[1] + 2, ez = br.hi[2] - br.lo[2] + 2;
  const int rows = ey * ez;
  const int lane = threadIdx.x & 63;
  const int wave = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int n_waves = (int)(gridDim.x * (blockDim.x >> 6));
  float mn = INFINITY, mx = -INFINITY;
  for (int r = wave; r < rows; r += n_waves) {
    const int y = r % ey, z = r / ey;
    for (int x = lane; x < ex; x += 64) {
      const float v = src_at<T>(s, br.lo[0] - 1 + x, br.lo[1] - 1 + y, br.lo[2] - 1 + z);
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, off));
    mx = fmaxf(mx, __shfl_xor(mx, off));
  }
  if (lane == 0 && mn <= mx) {
    atomicMin(&ctr->minmax[b][0], ordered_bits(mn));
    atomicMax(&ctr->minmax[b][1], ordered_bits(mx));
  }
}

__global__ void init_minmax_kernel(BcCounters* ctr, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    ctr->minmax[i][0] = 0xffffffffu;
    ctr->minmax[i][1] = 0u;
  }
}

// scale/offset of each brick from its stored range (FP32 formulas:
// o = (min+max)/2, s = (max-min)/896, s = 1 when max == min)
__global__ void finalize_kernel(BcBrick* bricks, const BcCounters* ctr, int first, int count, int storage) {
  const int b = first + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= first + count) return;
  const float mn = from_ordered(ctr->minmax[b][0]);
  const float mx = from_ordered(ctr->minmax[b][1]);
  bricks[b].vmin = mn;
  bricks[b].vmax = mx;
  float s = 1.0f, o = 0.0f;
  if (storage == 2) {
    if (mx == mn) {
      s = 1.0f;
      o = mn;
    } else {
      o = (mn + mx) / 2.0f;
      s = (mx - mn) / 896.0f;
    }
  }
  bricks[b].scale = s;
  bricks[b].offs = o;
  // the encodes below are monotone (round to nearest, saturating), so the
  // largest stored element is the encode of the largest source value; its
  // decode bounds every value the brick can produce (maximum intensity
  // projection stops a ray there)
  float dmax = mx;
  if (storage == 1) dmax = __half2float(__float2half_rn(mx));
  if (storage == 2) dmax = __builtin_fmaf(bc_e4m3_decode(bc_e4m3_encode((mx - o) * (1.0f / s))), s, o);
  bricks[b].dmax = dmax;
}

// encode + layout: brick first + blockIdx.y; a workgroup fills the row of
// micro-blocks (all x) at micro-block coordinates (y, z) = blockIdx.x, whose
// stored elements are contiguous: consecutive threads write consecutive
// elements, and a wave's reads fall on a dozen source rows
template <typename T, int FMT>
__global__ __launch_bounds__(256) void encode_kernel(SrcView s, const BcBrick* __restrict__ bricks, int first,
                                                     void* pool) {
  const BcBrick& br = bricks[first + (int)blockIdx.y];
  const int mb0 = br.mb[0], mb1 = br.mb[1];
  const int slabs = mb1 * br.mb[2];
  const int cx = br.hi[0] - br.lo[0], cy = br.hi[1] - br.lo[1], cz = br.hi[2] - br.lo[2];
  const float inv = 1.0f / br.scale, offs = br.offs;
  const int n_el = mb0 * BC_MB_ELEMS;
  for (int sl = (int)blockIdx.x; sl < slabs; sl += (int)gridDim.x) {
    const int mby = sl % mb1, mbz = sl / mb1;
    const int64_t base = br.offset + (int64_t)sl * n_el;
    for (int e = (int)threadIdx.x; e < n_el; e += (int)blockDim.x) {
      const int mbx = e / BC_MB_ELEMS, in = e - mbx * BC_MB_ELEMS;
      const int row = in / BC_ROW, wx = in - row * BC_ROW;   // the fifth repeats the next micro-block's first voxel
      // local ghosted index (0 <-> voxel lo-1); padding replicates the last ghost
      const int lx = min(mbx * 4 + wx, cx + 1);
      const int ly = min(mby * 4 + (row & 3), cy + 1);
      const int lz = min(mbz * 4 + (row >> 2), cz + 1);
      const float v = src_at<T>(s, br.lo[0] - 1 + lx, br.lo[1] - 1 + ly, br.lo[2] - 1 + lz);
      if (FMT == 0) {
        static_cast<float*>(pool)[base + e] = v;
      } else if (FMT == 1) {
        static_cast<__half*>(pool)[base + e] = __float2half_rn(v);
      } else {
        const float xq = (v - offs) * inv;
        static_cast<uint8_t*>(pool)[base + e] = bc_e4m3_encode(xq);
      }
    }
  }
}

inline SrcView make_src(const BcLoadSrc& s) {
  SrcView v;
  v.ptr = s.ptr;
  v.sx = s.strides[0]; v.sy = s.strides[1]; v.sz = s.strides[2];
  v.ox = s.origin[0]; v.oy = s.origin[1]; v.oz = s.origin[2];
  v.nx = s.dims[0]; v.ny = s.dims[1]; v.nz = s.dims[2];
  return v;
}

}  // namespace

hipError_t bc_launch_init_minmax(BcCounters* ctr, int n, hipStream_t st) {
  init_minmax_kernel<<<(n + 255) / 256, 256, 0, st>>>(ctr, n);
  return hipGetLastError();
}

hipError_t bc_launch_minmax(const BcLoadSrc& src, const BcBrick* bricks, int first, int count, int max_rows,
                            BcCounters* ctr, hipStream_t st) {
  SrcView s = make_src(src);
  const dim3 grid((unsigned)std::max(1, std::min((max_rows + 3) / 4, 64)), (unsigned)count);
  if (src.dtype == 0)
    minmax_kernel<float><<<grid, 256, 0, st>>>(s, bricks, first, ctr);
  else
    minmax_kernel<__half><<<grid, 256, 0, st>>>(s, bricks, first, ctr);
  return hipGetLastError();
}

hipError_t bc_launch_finalize(BcBrick* bricks, const BcCounters* ctr, int first, int count, int storage,
                              hipStream_t st) {
  finalize_kernel<<<(count + 255) / 256, 256, 0, st>>>(bricks, ctr, first, count, storage);
  return hipGetLastError();
}

hipError_t bc_launch_encode(const BcLoadSrc& src, const BcBrick* bricks, int first, int count, int64_t max_rows,
                            int storage, void* pool, hipStream_t st) {
  SrcView s = make_src(src);
  // one workgroup per row of micro-blocks (up to the largest brick's y * z count in micro-blocks)
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(max_rows, 65535)), (unsigned)count);
  if (src.dtype == 0) {
    if (storage == 0) encode_kernel<float, 0><<<grid, 256, 0, st>>>(s, bricks, first, pool);
    else if (storage == 1) encode_kernel<float, 1><<<grid, 256, 0, st>>>(s, bricks, first, pool);
    else encode_kernel<float, 2><<<grid, 256, 0, st>>>(s, bricks, first, pool);
  } else {
    if (storage == 0) encode_kernel<__half, 0><<<grid, 256, 0, st>>>(s, bricks, first, pool);
    else if (storage == 1) encode_kernel<__half, 1><<<grid, 256, 0, st>>>(s, bricks, first, pool);
    else encode_kernel<__half, 2><<<grid, 256, 0, st>>>(s, bricks, first, pool);
  }
  return hipGetLastError();
}
