// Ray casting of bricks into sub-images (the per-GPU ray-casting step of
// Sections 1.2 and 2.3.2) and the empty-space classification it uses.
//
//  classify  once per transfer-function table: one bit per interpolation cell
//            of every brick (the cube between 2x2x2 neighbouring stored
//            voxels) telling whether any value the cell can interpolate to
//            maps to a non-zero table entry.  A sample in a clear cell adds
//            exactly zero to its ray, so it is counted but not evaluated.
//            For maximum intensity projection a cell is clear when every
//            value it can take lies in the leading run of colour-map entries
//            equal to the first one: such a maximum, and every smaller one,
//            maps to that first entry, so it never changes the pixel.
//  render    persistent kernel: every wave pulls (brick, view, 8x8 tile) work
//            items from a device counter and casts the tile's 64 rays
//            through the brick: ray from the viewer's matrices, clipping to
//            the cube and the brick, samples at a fixed step anchored at the
//            cube entry, trilinear interpolation, transfer-function lookup,
//            front-to-back compositing with early ray termination.
//
// Sample positions.  Per ray and brick the first sample's brick-local
// position and the step vector are formed in double-float arithmetic and
// turned into 32.32 fixed point; every later sample position is an exact
// integer sum, so the cell index and the interpolation weights of sample j
// carry about 2^-32 voxels of error however far the ray has travelled.
//
// Lane schedule.  Each lane walks its own ray in chunks of 32 samples.  For a
// chunk it first gathers the 32 occupancy bits (cheap, all lanes in step),
// then evaluates only the samples whose cell is occupied, lowest first, so a
// lane's evaluations do not wait for the empty stretches of other lanes.
// FP32 compositing takes them two at a time: both samples' cells are
// gathered together (those gathers mostly miss the L1, so two in flight hide
// part of the wait), then the two are folded in order.
//
// Fewer gathers, fewer instructions.  The kernel is bound by the latency of
// its gathers (the L1 misses above all) together with instruction issue, not
// by HBM bandwidth.  So each lane avoids loads it can do without: consecutive
// samples in the same occupancy word reuse the word (the repeated load gets an
// out-of-range offset, answered by the range check without a cache access),
// and consecutive evaluated samples in the same interpolation cell reuse the
// cell's 8 voxels held in registers.  And the per-sample arithmetic is kept to
// single instructions where it can be: 24-bit multiply-adds with the strides
// in scalar registers, a floor-convert, a fract, a median-of-three clamp.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <float.h>
#include "bc_types.h"
#include "bc_kernels.h"
#include "bc_df.h"
#include "bc_e4m3.h"

// Launch data that no wave writes while the ray caster runs (frame inputs,
// view and brick records, the queue tables), addressed in the constant address
// space so that wave-uniform reads of it become scalar loads: they then wait on
// the scalar counter, not behind the vector loads and atomics in flight.
#define KC(T) const __attribute__((address_space(4))) T
template <typename T> __device__ __forceinline__ KC(T)* kc(const T* p) { return (KC(T)*)p; }

namespace {

// ------------------------------------------------------------------ storage
template <int FMT>
__device__ __forceinline__ float decode(uint32_t raw, float s, float o) {
  if (FMT == 0) return __uint_as_float(raw);
  if (FMT == 1) return __half2float(__ushort_as_half((unsigned short)raw));
  return __builtin_fmaf(bc_e4m3_decode(raw), s, o);
}

template <int FMT>
__device__ __forceinline__ float fetch(const void* __restrict__ pool, uint32_t idx, float s, float o) {
  if (FMT == 0) return decode<0>(__float_as_uint(static_cast<const float*>(pool)[idx]), s, o);
  if (FMT == 1) return decode<1>(static_cast<const uint16_t*>(pool)[idx], s, o);
  return decode<2>(static_cast<const uint8_t*>(pool)[idx], s, o);
}

// Buffer resources: the hardware range check turns an offset outside the
// brick (or its occupancy bits) into a zero instead of a fault.  Base and size
// are made wave-uniform explicitly so that the resource lives in scalar
// registers (a resource the compiler cannot prove uniform is rebuilt lane by
// lane around every load).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* ub = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

// a voxel and its +x neighbour (the next element) at a byte offset inside
// the brick, with one load
template <int FMT>
__device__ __forceinline__ void load_pair(__amdgpu_buffer_rsrc_t r, uint32_t ofs, float s, float o, float& a, float& b) {
  if (FMT == 0) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 p = __builtin_amdgcn_raw_buffer_load_b64(r, ofs, 0, 0);
    a = decode<0>(p.x, s, o);
    b = decode<0>(p.y, s, o);
  } else if (FMT == 1) {
    const uint32_t p = __builtin_amdgcn_raw_buffer_load_b32(r, ofs, 0, 0);
    a = decode<1>(p & 0xffffu, s, o);
    b = decode<1>(p >> 16, s, o);
  } else {
    // the hardware conversion of two E4M3 bytes is exact, as is the decode
    // above (the pool never holds the NaN codes: the encoder saturates)
    typedef float f2 __attribute__((ext_vector_type(2)));
    const uint32_t p = __builtin_amdgcn_raw_buffer_load_b16(r, ofs, 0, 0);
    const f2 v = __builtin_amdgcn_cvt_pk_f32_fp8((int)p, false);
    if (FMT == 3) {   // the codes' values only: the caller applies scale and offset
      a = v.x;
      b = v.y;
    } else {
      a = __builtin_fmaf(v.x, s, o);
      b = __builtin_fmaf(v.y, s, o);
    }
  }
}

// a * b + c on the low 24 bits of a and b (one multiply-add instruction)
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) { return __umul24(a, b) + c; }

// element index, inside the brick, of ghosted local voxel (x, y, z) >= 0:
// 4x4x4 micro-blocks stored row-major, each as 16 rows (y, then z) of 5
// elements, x fastest; element index + 1 is always the voxel at x + 1
__device__ __forceinline__ uint32_t vox_index(int x, int y, int z, int mbx, int mby) {
  const uint32_t blk = mad_u24(mad_u24((uint32_t)z >> 2, (uint32_t)mby, (uint32_t)y >> 2), (uint32_t)mbx,
                               (uint32_t)x >> 2);
  const uint32_t in_blk = mad_u24((uint32_t)(z & 3), 4u * BC_ROW, mad_u24((uint32_t)(y & 3), BC_ROW, (uint32_t)(x & 3)));
  return mad_u24(blk, BC_MB_ELEMS, in_blk);
}

// (a & mask) | (b & ~mask) in one instruction (the compiler splits the
// expression into ands and ors)
__device__ __forceinline__ uint32_t bfi_u32(uint32_t mask, uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(a), "v"(b));
  return r;
}

// a * b + c on signed 24-bit a and b (one multiply-add instruction)
__device__ __forceinline__ int mad_i24(int a, int b, int c) { return __mul24(a, b) + c; }

// floor(x) as an integer in one instruction
__device__ __forceinline__ int floor_i32(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// ------------------------------------------------------------------ classify
struct ClassifyArgs {
  const BcBrick* bricks;
  const BcFrameIn* fin;
  uint32_t* occ;
  const void* pool;
  int32_t n_bricks;
  int32_t max_words;      // largest occupancy word count of a brick
  int32_t mip;            // classify for maximum intensity projection
};

template <int FMT>
__global__ __launch_bounds__(256) void classify_kernel(ClassifyArgs a) {
  __shared__ int32_t nzp[BC_MAX_K + 1];   // nzp[k] = entries that matter among the first k
  __shared__ int32_t part[256];
  const int K = a.fin->K;
  const int tid = threadIdx.x;
  // block-wide prefix count of the entries that matter: non-zero opacity when
  // compositing (premultiplied colour is zero wherever opacity is), different
  // from the first entry for maximum intensity projection
  const float4* tab = reinterpret_cast<const float4*>(a.fin->table);
  const float4 e0 = tab[0];
  auto matters = [&](int k) -> int {
    const float4 e = tab[k];
    if (!a.mip) return e.w != 0.0f;
    return e.x != e0.x || e.y != e0.y || e.z != e0.z || e.w != e0.w;
  };
  const int per = (K + 255) / 256;
  int cnt = 0;
  for (int k = tid * per; k < min(K, (tid + 1) * per); ++k) cnt += matters(k);
  part[tid] = cnt;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < 256; ++i) { const int t = part[i]; part[i] = run; run += t; }
  }
  __syncthreads();
  int run = part[tid];
  for (int k = tid * per; k < min(K, (tid + 1) * per); ++k) {
    nzp[k] = run;
    run += matters(k);
  }
  if (tid == 255) nzp[K] = run;
  __syncthreads();
  const float sc = a.fin->tf_scale, bi = a.fin->tf_bias, kmax = (float)(K - 1);

  const int64_t total = (int64_t)a.n_bricks * a.max_words;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + tid; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(g / a.max_words);
    const int w = (int)(g % a.max_words);
    const BcBrick& br = a.bricks[b];
    const int WX = br.occ_w[0], WY = br.occ_w[1], WZ = br.occ_w[2];
    if (w >= WX * WY * WZ) continue;
    const int wx = w % WX, wy = (w / WX) % WY, wz = w / (WX * WY);
    // cells 0..ncell-1 per axis; cell i spans ghosted voxels i and i+1
    const int ncx = br.hi[0] - br.lo[0] + 1, ncy = br.hi[1] - br.lo[1] + 1, ncz = br.hi[2] - br.lo[2] + 1;
    const int vmax_x = ncx, vmax_y = ncy, vmax_z = ncz;   // last ghosted voxel index
    float v[3][5][5];
    const float s_q = br.scale, o_q = br.offs;
    // FP8 compositing: the ray caster interpolates the codes' values and maps
    // the result to the table with the brick's scale and offset folded in,
    // fma(q, scale * s, fma(o, scale, bias)); the cells are bounded through
    // the same mapping of the same values, so that every index the ray caster
    // can form lies inside the checked range
    const bool fold = FMT == 2 && !a.mip;
    const float csc = fold ? sc * s_q : sc, cbi = fold ? __builtin_fmaf(o_q, sc, bi) : bi;
    const float ds = fold ? 1.0f : s_q, dof = fold ? 0.0f : o_q;
    const void* pool = static_cast<const char*>(a.pool) + br.offset * (FMT == 0 ? 4 : (FMT == 1 ? 2 : 1));
    for (int z = 0; z < 3; ++z)
      for (int y = 0; y < 5; ++y)
        for (int x = 0; x < 5; ++x) {
          const int gx = clampi(wx * 4 + x, 0, vmax_x), gy = clampi(wy * 4 + y, 0, vmax_y),
                    gz = clampi(wz * 2 + z, 0, vmax_z);
          v[z][y][x] = fetch<FMT>(pool, vox_index(gx, gy, gz, br.mb[0], br.mb[1]), ds, dof);
        }
    uint32_t bits = 0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 4; ++cy)
        for (int cx = 0; cx < 4; ++cx) {
          if (wx * 4 + cx >= ncx || wy * 4 + cy >= ncy || wz * 2 + cz >= ncz) continue;
          float lo = FLT_MAX, hi = -FLT_MAX;
          for (int c = 0; c < 8; ++c) {
            const float t = v[cz + (c >> 2)][cy + ((c >> 1) & 1)][cx + (c & 1)];
            lo = fminf(lo, t);
            hi = fmaxf(hi, t);
          }
          // trilinear values lie within the corner range up to a few roundings
          const float m = fmaxf(fabsf(lo), fabsf(hi)) * 9.5367431640625e-07f + 1e-30f;   // 2^-20
          float xl = __builtin_fmaf(lo - m, csc, cbi), xh = __builtin_fmaf(hi + m, csc, cbi);
          xl = fminf(fmaxf(xl, 0.0f), kmax);
          xh = fminf(fmaxf(xh, 0.0f), kmax);
          const int il = a.mip ? 0 : min((int)xl, K - 2), ih = min((int)xh, K - 2) + 1;
          if (nzp[ih + 1] - nzp[il] > 0) bits |= 1u << ((cz << 4) | (cy << 2) | cx);
        }
    a.occ[br.occ_offset + w] = bits;
  }
}

// ------------------------------------------------------------------ rays
__device__ __forceinline__ df dfv(float hi, float lo) { return df_make(hi, lo); }

// smallest j >= 0 with t_in + (j + 1/2) dt >= t, that is ceil(q - 1/2) for
// q = (t - t_in) / dt, taken exactly from the double-float q: q.hi - 1/2 is
// exact (q stays below 2^22: the boundary refuses steps with more samples
// along the cube's diagonal), and unless it is an integer the trailing part
// (below half its ulp) cannot carry it past one
__device__ __forceinline__ int first_index(df t_in, df idt, df t) {
  const df q = df_mul(df_sub(t, t_in), idt);
  const float c = q.hi - 0.5f;
  const float j = ceilf(c);
  return (int)fmaxf((j == c && q.lo > 0.0f) ? j + 1.0f : j, 0.0f);
}

struct Slab { df t0, t1; bool miss; };

// slab test with the reciprocal direction (id[a] valid where d[a] != 0)
__device__ __forceinline__ Slab slab_df(const df* o, const df* d, const df* id, const float* lo, const float* hi) {
  Slab s;
  s.t0 = df_from(-INFINITY);
  s.t1 = df_from(INFINITY);
  s.miss = false;
  for (int a = 0; a < 3; ++a) {
    if (d[a].hi == 0.0f && d[a].lo == 0.0f) {
      const bool in = df_ge(o[a], df_from(lo[a])) && df_lt(o[a], df_from(hi[a]));
      if (!in) s.miss = true;
      continue;
    }
    const df ta = df_mul(df_add_f(df_neg(o[a]), lo[a]), id[a]);
    const df tb = df_mul(df_add_f(df_neg(o[a]), hi[a]), id[a]);
    s.t0 = df_max(s.t0, df_min(ta, tb));
    s.t1 = df_min(s.t1, df_max(ta, tb));
  }
  return s;
}

// 32.32 fixed point of a double-float (each part truncated; error < 2^-31)
__device__ __forceinline__ int64_t q32(df a) {
  return (int64_t)(a.hi * 4294967296.0f) + (int64_t)(a.lo * 4294967296.0f);
}

struct RaySeg {
  int n;                 // samples of the ray inside the brick
  int64_t u[3];          // first sample, ghosted brick-local coordinate minus 1/2, 32.32
  int64_t s[3];          // step vector, 32.32
};

__device__ __forceinline__ df df_abs(df a) { return df_lt(a, df_from(0.0f)) ? df_neg(a) : a; }

// Ray of pixel (px, py) against brick br: the samples t_j = t_in + (j+1/2) dt
// of the ray's cube interval that fall in the brick's half-open box.  The step
// is the view's, or with the per-voxel policy 1 / max_a |d_a| (consecutive
// samples one voxel apart along the ray's dominant axis, the discrete ray
// casting of Section 2.3.2).
__device__ bool ray_segment(KC(BcViewParams)& vp, const int32_t* gdims, KC(BcBrick)& br, int px, int py,
                            bool per_voxel, RaySeg& seg) {
  const int W = vp.width, H = vp.height;
  const df x = df_mul_f(dfv(vp.iw_hi, vp.iw_lo), (float)(2 * px + 1 - W));
  const df y = df_mul_f(dfv(vp.ih_hi, vp.ih_lo), (float)(H - 2 * py - 1));
  df o[3], d[3], id[3];
  if (vp.kind == 0) {
    df u[3];
    for (int a = 0; a < 3; ++a) {
      o[a] = dfv(vp.e_hi[a], vp.e_lo[a]);
      u[a] = df_add(df_add(df_mul(dfv(vp.a_hi[a], vp.a_lo[a]), x), df_mul(dfv(vp.b_hi[a], vp.b_lo[a]), y)),
                    dfv(vp.c_hi[a], vp.c_lo[a]));
    }
    const df len = df_sqrt(df_add(df_add(df_mul(u[0], u[0]), df_mul(u[1], u[1])), df_mul(u[2], u[2])));
    const df ilen = df_div(df_from(1.0f), len);
    for (int a = 0; a < 3; ++a) d[a] = df_mul(u[a], ilen);
  } else {
    for (int a = 0; a < 3; ++a) {
      o[a] = df_add(df_add(dfv(vp.e_hi[a], vp.e_lo[a]), df_mul(dfv(vp.a_hi[a], vp.a_lo[a]), x)),
                    df_mul(dfv(vp.b_hi[a], vp.b_lo[a]), y));
      d[a] = dfv(vp.c_hi[a], vp.c_lo[a]);
    }
  }
  for (int a = 0; a < 3; ++a)
    id[a] = (d[a].hi == 0.0f && d[a].lo == 0.0f) ? df_from(0.0f) : df_div(df_from(1.0f), d[a]);
  const float zero3[3] = {0.0f, 0.0f, 0.0f};
  const float N3[3] = {(float)gdims[0], (float)gdims[1], (float)gdims[2]};
  const Slab g = slab_df(o, d, id, zero3, N3);
  const df t_in = df_max(df_from(0.0f), g.t0);
  if (g.miss || !df_lt(t_in, g.t1)) return false;
  const float blo[3] = {(float)br.lo[0], (float)br.lo[1], (float)br.lo[2]};
  const float bhi[3] = {(float)br.hi[0], (float)br.hi[1], (float)br.hi[2]};
  const Slab b = slab_df(o, d, id, blo, bhi);
  if (b.miss || !df_lt(b.t0, b.t1)) return false;
  df dt = dfv(vp.dt_hi, vp.dt_lo), idt = dfv(vp.idt_hi, vp.idt_lo);
  if (per_voxel) {
    idt = df_max(df_max(df_abs(d[0]), df_abs(d[1])), df_abs(d[2]));
    dt = df_div(df_from(1.0f), idt);
  }
  const int n = first_index(t_in, idt, g.t1);
  int j0 = (b.t0.hi == -INFINITY) ? 0 : first_index(t_in, idt, b.t0);
  int j1 = (b.t1.hi == INFINITY) ? n : first_index(t_in, idt, b.t1);
  j0 = min(j0, n);
  j1 = min(max(j1, j0), n);
  if (j1 <= j0) return false;
  seg.n = j1 - j0;
  const df t0 = df_add(t_in, df_mul_f(dt, (float)j0 + 0.5f));
  for (int a = 0; a < 3; ++a) {
    const df p = df_add(o[a], df_mul(t0, d[a]));
    seg.u[a] = q32(df_add_f(p, 0.5f - (float)br.lo[a]));
    seg.s[a] = q32(df_mul(dt, d[a]));
  }
  return true;
}

__device__ __forceinline__ int hi32(int64_t v) { return (int)(v >> 32); }
__device__ __forceinline__ float frac32(int64_t v) { return (float)(uint32_t)v * 2.3283064365386963e-10f; }

// ------------------------------------------------------------------ render
// OP 0: front-to-back compositing into premultiplied RGBA with early
// termination at opacity tau.  OP 1: maximum intensity projection, the largest
// sample value per ray (-inf for a ray with no sample in the brick, -FLT_MAX
// when all its samples fell in clear cells), stopping once it reaches the
// largest value the brick stores.
// URGENT: the waves issue at the raised priority levels (2, and 3 while they
// evaluate occupied samples) instead of the base levels (0 and 1): the plain
// passes' setting, while a pass that runs beside a more urgent one (a learned
// frame's coarse pass beside its validation pass) keeps the base levels; a
// template parameter so that each instantiation holds one setting.
template <int FMT, bool TF_LDS, int CHUNK, int OP, bool URGENT>
__global__ __launch_bounds__(256, 4) void render_kernel(BcFramePtrs f) {
  // table entry k at 2k, its difference to entry k+1 at 2k+1
  __shared__ float4 s_tab[(TF_LDS && OP == 0) ? 2 * BC_TF_LDS : 2];
  const int lane = threadIdx.x & 63;
  KC(BcFrameIn)* fin = kc(f.fin);
  KC(BcCounters)* cr = kc(f.ctr);   // the lines the waves read, not the queue counters
  if (cr->n_items == 0) return;   // e.g. a conditional pass that is not needed
  if (URGENT) __builtin_amdgcn_s_setprio(2);
  const int K = fin->K;
  const float tf_scale = fin->tf_scale;
  // held in a vector register: an FMA can read only one scalar operand
  float tf_bias = fin->tf_bias;
  if (OP == 0) asm volatile("" : "+v"(tf_bias));
  const float kmax_f = (float)(K - 1);
  const float4* gtab = reinterpret_cast<const float4*>(f.fin->table);   // gathered per lane
  if (TF_LDS && OP == 0) {
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const float4 a = gtab[k], b = gtab[min(k + 1, K - 1)];
      s_tab[2 * k] = a;
      s_tab[2 * k + 1] = make_float4(b.x - a.x, b.y - a.y, b.z - a.z, b.w - a.w);
    }
    __syncthreads();
  }

  const int nv = f.n_views, nb = f.n_bricks;
  const int KB = nb * nv;
  const uint32_t n_items = cr->n_items;
  const bool ess = f.ess != 0;
  const bool per_voxel = f.step_policy != 0;
  const int ts = fin->tile_stride;
  constexpr uint32_t esz = FMT == 0 ? 4 : (FMT == 1 ? 2 : 1);
  // per-lane sample counts (a lane takes at most a few thousand samples per
  // item and a few dozen items per launch, far below 2^32)
  uint32_t nominal = 0, evaluated = 0;
  // the queue of the XCD this workgroup runs on first, then the others once
  // it is drained; the XCD comes from its hardware id register (XCC_ID, bits
  // 0-3), not from the block index, so that the choice holds however the
  // dispatcher deals workgroups to the XCDs (0.2% faster on the bench orbit).
  // Q is 8 or 1, so Q - 1 masks the id to a queue (written without a branch,
  // which left the projection kernels out of scalar registers)
  const int Q = (int)cr->n_queues;
  int q = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & (uint32_t)(Q - 1)), drained = 0;
  uint32_t q_lo = cr->qbound[q], q_hi = cr->qbound[q + 1];
  // a slot is claimed when the wave needs it: claiming one item ahead, the
  // atomic in flight during the item before, made the launch 8% slower
  for (;;) {
    uint32_t item = 0;
    bool have = false;
    while (drained < Q) {
      const uint32_t claim = lane == 0 ? atomicAdd(&f.ctr->q[q].next, 1u) : 0u;
      const uint32_t it = q_lo + (uint32_t)__builtin_amdgcn_readlane((int)claim, 0);
      if (it < q_hi && it < n_items) {
        item = it;
        have = true;
        break;
      }
      ++drained;
      q = (q + 1 == Q) ? 0 : q + 1;
      q_lo = cr->qbound[q];
      q_hi = cr->qbound[q + 1];
    }
    if (!have) break;
    KC(int32_t)* perm = kc(f.item_perm);
    int lo = 0, hi = KB;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((uint32_t)perm[mid] <= item) lo = mid; else hi = mid;
    }
    KC(int4)& ent = kc(f.item_entry)[lo];
    const int b = ent.x & 0xffff, v = ent.x >> 16, cx = ent.y;
    const int local = (int)(item - (uint32_t)perm[lo]);
    const int tx = ent.z + (local % cx) * ts, ty = ent.w + (local / cx) * ts;
    KC(BcViewParams)& vp = kc(f.views)[v];
    const int tsh = f.tile_shift;
    const int px = (tx << tsh) + (lane & ((1 << tsh) - 1));
    const int py = ty * (64 >> tsh) + (lane >> tsh);
    KC(BcBrick)& br = kc(f.bricks)[b];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    float mx = -INFINITY;
    RaySeg seg;
    if (px < vp.width && py < vp.height && ray_segment(vp, f.gdims, br, px, py, per_voxel, seg)) {
      const float tau = vp.tau;
      const float bound = br.dmax;
      mx = -FLT_MAX;
      const int cmx = br.hi[0] - br.lo[0], cmy = br.hi[1] - br.lo[1], cmz = br.hi[2] - br.lo[2];
      const int mbx = br.mb[0], mby = br.mb[1];
      const uint32_t WX = (uint32_t)br.occ_w[0], WY = (uint32_t)br.occ_w[1], WX4 = 4u * WX;
      const uint32_t n_occ = WX * WY * (uint32_t)br.occ_w[2];
      const __amdgpu_buffer_rsrc_t occ = make_rsrc(f.occ + br.occ_offset, n_occ * 4u);
      const uint32_t n_vox = (uint32_t)br.mb[0] * (uint32_t)br.mb[1] * (uint32_t)br.mb[2] * BC_MB_ELEMS;
      const __amdgpu_buffer_rsrc_t pool = make_rsrc(static_cast<const char*>(f.pool) + br.offset * esz, n_vox * esz);
      const float s_q = br.scale, o_q = br.offs;
      // FP8 compositing: interpolation is linear, so the brick's scale and
      // offset move from the 8 decoded voxels into the table index (one
      // multiply-add per sample); MIP compares decoded values with the
      // brick maximum and decodes each voxel
      constexpr bool FOLD = FMT == 2 && OP == 0;
      // FP32 evaluates its occupied samples two at a time (its gathers miss
      // the L1 most; 1.305 -> 1.229 ms on the bench orbit, and 0.915 -> 0.879
      // ms with maximum intensity projection at the per-voxel step); the
      // narrower forms, whose cells more often share cached lines, one at a
      // time, and so does projection with 64-sample chunks, which would spill
      constexpr bool PAIRS = FMT == 0 && (OP == 0 || CHUNK == 32);
      const float tsc = FOLD ? tf_scale * s_q : tf_scale, tbi = FOLD ? __builtin_fmaf(o_q, tf_scale, tf_bias) : tf_bias;
      // byte steps to the +y/+z neighbour: inside a micro-block, or across
      // into the next one (from its last row or slice)
      constexpr uint32_t sh = FMT == 0 ? 2 : (FMT == 1 ? 1 : 0);
      uint32_t dyb = ((uint32_t)mbx * BC_MB_ELEMS - 3u * BC_ROW) << sh,
               dzb = ((uint32_t)mbx * (uint32_t)mby * BC_MB_ELEMS - 12u * BC_ROW) << sh;
      if (OP == 0) asm volatile("" : "+v"(dyb), "+v"(dzb));   // (selected per lane below)
      // the element index of vox_index as a sum of per-axis terms: along x
      // 80 (x>>2) + (x&3) = 20 x - 19 (x&3), along y and z likewise with the
      // micro-block row and slice strides; in bytes
      const uint32_t cxb = 20u << sh, cyb = (20u * (uint32_t)mbx) << sh, czb = (20u * (uint32_t)mbx * (uint32_t)mby) << sh;
      const int rxb = -(int)(19u << sh), ryb = (int)(BC_ROW << sh) - (int)cyb, rzb = (int)((4u * BC_ROW) << sh) - (int)czb;
      int64_t uc0 = seg.u[0], uc1 = seg.u[1], uc2 = seg.u[2];
      // the step, with y and z scaled by 4 and 16 (kept only so, to save
      // registers) so that in the occupancy pass bits 2-3 of the integer part
      // of y' hold y%4 and bit 4 of z' holds z%2
      const int64_t s0 = seg.s[0], s1q = seg.s[1] * 4, s2q = seg.s[2] * 16;
      const float sfx = (float)s0 * 2.3283064365386963e-10f, sfy = (float)seg.s[1] * 2.3283064365386963e-10f,
                  sfz = (float)seg.s[2] * 2.3283064365386963e-10f;
      int used = seg.n;
      // the voxels of the cell the lane interpolated last, and its offset
      // (none yet)
      uint32_t cell_ofs = 0xffffffffu;
      float cv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < seg.n; k += CHUNK) {
        const int cnt = min(CHUNK, seg.n - k);
        uint64_t mask = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
        if (ess) {
          int64_t un0 = uc0, un1 = uc1 * 4, un2 = uc2 * 16;
          // occupancy bits of the chunk's samples (cells outside the brick
          // read as clear through the buffer range check)
          // all addresses first, then all loads in flight together
          uint64_t m = 0;
          uint32_t occ_ofs = 0xffffffffu, occ_word = 0u;   // the occupancy word loaded last
#pragma unroll
          for (int h = 0; h < CHUNK / 8; ++h) {
            uint32_t wofs[8], bit[8], word[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              // x, 4 y + (2 bits), 16 z + (4 bits)
              const uint32_t ix = (uint32_t)hi32(un0), iy4 = (uint32_t)hi32(un1), iz16 = (uint32_t)hi32(un2);
              // word (x/4, y/4, z/2) as a byte offset; bit (x%4) + 4 (y%4) + 16 (z%2), of
              // which the bit-field extract below reads only the low five bits
              wofs[i] = mad_u24(mad_u24(iz16 >> 5, WY, iy4 >> 4), WX4, ix & ~3u);
              // two bit-field inserts: x%4 into 4 (y%4), then into 16 (z%2)
              bit[i] = bfi_u32(15u, bfi_u32(3u, ix, iy4), iz16);
              un0 += s0; un1 += s1q; un2 += s2q;
            }
            // a sample in the same word as the one before it reuses that
            // word: its load gets an offset past the end of the bits, which
            // the range check answers without a cache access
            bool fresh[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) fresh[i] = wofs[i] != (i ? wofs[i - 1] : occ_ofs);
            occ_ofs = wofs[7];
#pragma unroll
            for (int i = 0; i < 8; ++i)
              word[i] = __builtin_amdgcn_raw_buffer_load_b32(occ, fresh[i] ? wofs[i] : 0xfffffff0u, 0, 0);
            uint32_t mh = 0;
            // (a reused sample's load returned zero: keep the word before)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              occ_word = word[i] | (fresh[i] ? 0u : occ_word);
              mh |= __builtin_amdgcn_ubfe(occ_word, bit[i], 1u) << i;
            }
            m |= (uint64_t)mh << (8 * h);
          }
          mask &= m;
        }
        bool stop = false;
        if (mask) {
          // a wave evaluating samples waits on dependent gathers; letting it
          // issue ahead of the waves gathering occupancy bits (whose loads are
          // all in flight together) shortens the frame
          __builtin_amdgcn_s_setprio(URGENT ? 3 : 1);
          // sample positions inside the chunk in FP32, relative to the
          // chunk's first sample: integer cell of that sample plus a
          // fraction that stays below 1 + CHUNK/2 voxels
          const int bx = hi32(uc0), by = hi32(uc1), bz = hi32(uc2);
          const float fx0 = frac32(uc0), fy0 = frac32(uc1), fz0 = frac32(uc2);
          // the sample that ended the ray (the loop runs out instead of
          // breaking, which keeps the loop's registers in place)
          int last = CHUNK - 1;
          for (int half = 0; half < CHUNK / 32; ++half) {
            uint32_t m32 = stop ? 0u : (uint32_t)(mask >> (32 * half));
            if constexpr (PAIRS) {
              // occupied samples two at a time: both cells' gathers in flight
              // together (the second sample's only if its cell differs from the
              // first's), then the samples folded in order; the arithmetic of
              // each sample is that of one taken alone
              while (m32) {
                const int i0 = 32 * half + (int)__builtin_ctz(m32);
                m32 &= m32 - 1u;
                const bool two = m32 != 0u;
                const int i1 = two ? 32 * half + (int)__builtin_ctz(m32) : i0;
                if (two) m32 &= m32 - 1u;
                float w0[3], w1[3];
                uint32_t a0, a1;
                int ry0, rz0, ry1, rz1;
                auto cell = [&](int i, float* w, uint32_t& a, int& ry, int& rz) {
                  const float fi = (float)i;
                  const float ux = __builtin_fmaf(fi, sfx, fx0), uy = __builtin_fmaf(fi, sfy, fy0),
                              uz = __builtin_fmaf(fi, sfz, fz0);
                  w[0] = __builtin_amdgcn_fractf(ux);
                  w[1] = __builtin_amdgcn_fractf(uy);
                  w[2] = __builtin_amdgcn_fractf(uz);
                  const uint32_t ix = (uint32_t)(bx + floor_i32(ux)), iy = (uint32_t)(by + floor_i32(uy)),
                                 iz = (uint32_t)(bz + floor_i32(uz));
                  ry = (int)(iy & 3u);
                  rz = (int)(iz & 3u);
                  a = (uint32_t)mad_i24(rz, rzb, mad_i24(ry, ryb, mad_i24((int)(ix & 3u), rxb,
                                        (int)mad_u24(ix, cxb, mad_u24(iy, cyb, __umul24(iz, czb))))));
                };
                auto gather = [&](uint32_t a, int ry, int rz, float* v) {
                  const uint32_t dy = ry == 3 ? dyb : (BC_ROW << sh);
                  const uint32_t dz = rz == 3 ? dzb : ((4u * BC_ROW) << sh);
                  const uint32_t a010 = a + dy, a001 = a + dz, a011 = a001 + dy;
                  load_pair<FOLD ? 3 : FMT>(pool, a, s_q, o_q, v[0], v[1]);
                  load_pair<FOLD ? 3 : FMT>(pool, a010, s_q, o_q, v[2], v[3]);
                  load_pair<FOLD ? 3 : FMT>(pool, a001, s_q, o_q, v[4], v[5]);
                  load_pair<FOLD ? 3 : FMT>(pool, a011, s_q, o_q, v[6], v[7]);
                };
                cell(i0, w0, a0, ry0, rz0);
                cell(i1, w1, a1, ry1, rz1);
                if (a0 != cell_ofs) {
                  gather(a0, ry0, rz0, cv);
                  cell_ofs = a0;
                }
                float cw[8];
                const bool own1 = two && a1 != a0;
                if (own1) gather(a1, ry1, rz1, cw);
                auto sample = [&](const float* v, const float* w, int i) {
                  const float c00 = __builtin_fmaf(w[0], v[1] - v[0], v[0]);
                  const float c10 = __builtin_fmaf(w[0], v[3] - v[2], v[2]);
                  const float c01 = __builtin_fmaf(w[0], v[5] - v[4], v[4]);
                  const float c11 = __builtin_fmaf(w[0], v[7] - v[6], v[6]);
                  const float c0 = __builtin_fmaf(w[1], c10 - c00, c00);
                  const float c1 = __builtin_fmaf(w[1], c11 - c01, c01);
                  const float val = __builtin_fmaf(w[2], c1 - c0, c0);
                  if (OP == 1) {
                    mx = fmaxf(mx, val);
                    if (mx >= bound) {
                      last = i;
                      stop = true;
                      m32 = 0u;
                    }
                    return;
                  }
                  const float xt = __builtin_amdgcn_fmed3f(__builtin_fmaf(val, tsc, tbi), 0.0f, kmax_f);
                  const int it = TF_LDS ? (int)xt : min((int)xt, K - 2);
                  const float ft = TF_LDS ? __builtin_amdgcn_fractf(xt) : xt - (float)it;
                  float4 q0, dq;
                  if (TF_LDS) {
                    q0 = s_tab[2 * it];
                    dq = s_tab[2 * it + 1];
                  } else {
                    q0 = gtab[it];
                    const float4 q1 = gtab[it + 1];
                    dq = make_float4(q1.x - q0.x, q1.y - q0.y, q1.z - q0.z, q1.w - q0.w);
                  }
                  const float om = 1.0f - acc.w;
                  acc.x = __builtin_fmaf(om, __builtin_fmaf(ft, dq.x, q0.x), acc.x);
                  acc.y = __builtin_fmaf(om, __builtin_fmaf(ft, dq.y, q0.y), acc.y);
                  acc.z = __builtin_fmaf(om, __builtin_fmaf(ft, dq.z, q0.z), acc.z);
                  acc.w = __builtin_fmaf(om, __builtin_fmaf(ft, dq.w, q0.w), acc.w);
                  if (acc.w >= tau) {
                    last = i;
                    stop = true;
                    m32 = 0u;
                  }
                };
                sample(cv, w0, i0);
                if (two && !stop) {
                  if (own1) {
  #pragma unroll
                    for (int q = 0; q < 8; ++q) cv[q] = cw[q];
                    cell_ofs = a1;
                  }
                  sample(cv, w1, i1);
                }
              }
            } else {
              while (m32) {
                const int i = 32 * half + (int)__builtin_ctz(m32);
                m32 &= m32 - 1u;
                const float fi = (float)i;
                const float ux = __builtin_fmaf(fi, sfx, fx0), uy = __builtin_fmaf(fi, sfy, fy0),
                            uz = __builtin_fmaf(fi, sfz, fz0);
                const float wx = __builtin_amdgcn_fractf(ux), wy = __builtin_amdgcn_fractf(uy),
                            wz = __builtin_amdgcn_fractf(uz);
                // the sample's cell (inside the brick: 0 <= ix, iy, iz < 2^24)
                const uint32_t ix = (uint32_t)(bx + floor_i32(ux)), iy = (uint32_t)(by + floor_i32(uy)),
                               iz = (uint32_t)(bz + floor_i32(uz));
                const int ry = (int)(iy & 3u), rz = (int)(iz & 3u);
                const uint32_t a000 = (uint32_t)mad_i24(
                    rz, rzb, mad_i24(ry, ryb, mad_i24((int)(ix & 3u), rxb,
                                                      (int)mad_u24(ix, cxb, mad_u24(iy, cyb, __umul24(iz, czb))))));
                // the 8 voxels of the sample's cell, loaded only when the cell
                // differs from the one the lane interpolated last
                if (a000 != cell_ofs) {
                  const uint32_t dy = ry == 3 ? dyb : (BC_ROW << sh);
                  const uint32_t dz = rz == 3 ? dzb : ((4u * BC_ROW) << sh);
                  const uint32_t a010 = a000 + dy, a001 = a000 + dz, a011 = a001 + dy;
                  load_pair<FOLD ? 3 : FMT>(pool, a000, s_q, o_q, cv[0], cv[1]);
                  load_pair<FOLD ? 3 : FMT>(pool, a010, s_q, o_q, cv[2], cv[3]);
                  load_pair<FOLD ? 3 : FMT>(pool, a001, s_q, o_q, cv[4], cv[5]);
                  load_pair<FOLD ? 3 : FMT>(pool, a011, s_q, o_q, cv[6], cv[7]);
                  cell_ofs = a000;
                }
                const float c00 = __builtin_fmaf(wx, cv[1] - cv[0], cv[0]);
                const float c10 = __builtin_fmaf(wx, cv[3] - cv[2], cv[2]);
                const float c01 = __builtin_fmaf(wx, cv[5] - cv[4], cv[4]);
                const float c11 = __builtin_fmaf(wx, cv[7] - cv[6], cv[6]);
                const float c0 = __builtin_fmaf(wy, c10 - c00, c00);
                const float c1 = __builtin_fmaf(wy, c11 - c01, c01);
                const float val = __builtin_fmaf(wz, c1 - c0, c0);
                if (OP == 1) {
                  mx = fmaxf(mx, val);
                  if (mx >= bound) {
                    last = i;
                    stop = true;
                    m32 = 0u;
                  }
                  continue;
                }
                // clamp to [0, K-1] (the median of three, exact)
                const float xt = __builtin_amdgcn_fmed3f(__builtin_fmaf(val, tsc, tbi), 0.0f, kmax_f);
                // (the table in LDS has an entry K-1 with a zero difference)
                const int it = TF_LDS ? (int)xt : min((int)xt, K - 2);
                const float ft = TF_LDS ? __builtin_amdgcn_fractf(xt) : xt - (float)it;
                // table entry and its difference to the next entry
                float4 q0, dq;
                if (TF_LDS) {
                  q0 = s_tab[2 * it];
                  dq = s_tab[2 * it + 1];
                } else {
                  q0 = gtab[it];
                  const float4 q1 = gtab[it + 1];
                  dq = make_float4(q1.x - q0.x, q1.y - q0.y, q1.z - q0.z, q1.w - q0.w);
                }
                const float om = 1.0f - acc.w;
                acc.x = __builtin_fmaf(om, __builtin_fmaf(ft, dq.x, q0.x), acc.x);
                acc.y = __builtin_fmaf(om, __builtin_fmaf(ft, dq.y, q0.y), acc.y);
                acc.z = __builtin_fmaf(om, __builtin_fmaf(ft, dq.z, q0.z), acc.z);
                acc.w = __builtin_fmaf(om, __builtin_fmaf(ft, dq.w, q0.w), acc.w);
                if (acc.w >= tau) {
                  last = i;
                  stop = true;
                  m32 = 0u;
                }
              }
            }
          }
          __builtin_amdgcn_s_setprio(URGENT ? 2 : 0);
          // the occupied samples up to the last one evaluated
          evaluated += (uint32_t)__builtin_popcountll(mask & (~0ull >> (63 - last)));
          if (stop) used = k + last + 1;
        }
        if (stop) break;
        uc0 += CHUNK * s0; uc1 += (CHUNK * s1q) >> 2; uc2 += (CHUNK * s2q) >> 4;
      }
      nominal += (uint32_t)used;
    }
    if (OP == 0) f.sub[(int64_t)item * 64 + lane] = acc;
    else reinterpret_cast<float*>(f.sub)[(int64_t)item * 64 + lane] = mx;
  }
  uint64_t wave_nominal = nominal, wave_evaluated = evaluated;
  for (int off = 32; off > 0; off >>= 1) {
    wave_nominal += __shfl_xor(wave_nominal, off);
    wave_evaluated += __shfl_xor(wave_evaluated, off);
  }
  if (lane == 0 && wave_nominal) {
    atomicAdd(&f.ctr->nominal, (unsigned long long)wave_nominal);
    atomicAdd(&f.ctr->evaluated, (unsigned long long)wave_evaluated);
  }
}

template <int FMT>
hipError_t launch_render_fmt(const BcFramePtrs& f, int n_workgroups, hipStream_t st) {
  const bool lds = f.K <= BC_TF_LDS;
  if (f.op == 1) {
    // the colour map is applied after the merge: no table in the ray caster
    if (f.chunk == 32) render_kernel<FMT, false, 32, 1, false><<<n_workgroups, 256, 0, st>>>(f);
    else render_kernel<FMT, false, 64, 1, false><<<n_workgroups, 256, 0, st>>>(f);
  } else if (f.chunk == 32) {
    if (lds && f.urgent) render_kernel<FMT, true, 32, 0, true><<<n_workgroups, 256, 0, st>>>(f);
    else if (lds) render_kernel<FMT, true, 32, 0, false><<<n_workgroups, 256, 0, st>>>(f);
    else render_kernel<FMT, false, 32, 0, false><<<n_workgroups, 256, 0, st>>>(f);
  } else {
    if (lds && f.urgent) render_kernel<FMT, true, 64, 0, true><<<n_workgroups, 256, 0, st>>>(f);
    else if (lds) render_kernel<FMT, true, 64, 0, false><<<n_workgroups, 256, 0, st>>>(f);
    else render_kernel<FMT, false, 64, 0, false><<<n_workgroups, 256, 0, st>>>(f);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t bc_launch_classify(const BcFramePtrs& f, int max_words, hipStream_t st) {
  ClassifyArgs a;
  a.bricks = f.bricks;
  a.fin = f.fin;
  a.occ = f.occ;
  a.pool = f.pool;
  a.n_bricks = f.n_bricks;
  a.max_words = max_words;
  a.mip = f.op == 1;
  const int64_t total = (int64_t)f.n_bricks * max_words;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
  if (f.storage == 0) classify_kernel<0><<<grid, 256, 0, st>>>(a);
  else if (f.storage == 1) classify_kernel<1><<<grid, 256, 0, st>>>(a);
  else classify_kernel<2><<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t bc_launch_render(const BcFramePtrs& f, int n_workgroups, hipStream_t st) {
  if (f.storage == 0) return launch_render_fmt<0>(f, n_workgroups, st);
  if (f.storage == 1) return launch_render_fmt<1>(f, n_workgroups, st);
  return launch_render_fmt<2>(f, n_workgroups, st);
}
