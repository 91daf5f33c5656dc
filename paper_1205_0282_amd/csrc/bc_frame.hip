// Per-frame kernels of the bricked ray caster.
//
//  setup     (FP64, one workgroup): inverse view transform, eye, per-brick
//            visibility keys and their sort, per-brick rendering rectangles
//            (Section 2.3.2, Figure 4) and the work-item prefix sums.
//  composite per pixel, folds the brick sub-images in visibility order with
//            "over" (Section 2.3.3; associativity of alpha blending).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <float.h>
#include "bc_types.h"
#include "bc_kernels.h"

namespace {

// ------------------------------------------------------------------ FP64 setup
__device__ void mat4_mul(const double* a, const double* b, double* c) {
#pragma clang fp contract(off)
  for (int r = 0; r < 4; ++r)
    for (int col = 0; col < 4; ++col) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s = s + a[r * 4 + k] * b[k * 4 + col];
      c[r * 4 + col] = s;
    }
}

// Gauss-Jordan inverse with partial pivoting (row-major); false if singular
__device__ bool mat4_inv(const double* m, double* inv) {
#pragma clang fp contract(off)
  double a[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      a[r][c] = m[r * 4 + c];
      a[r][c + 4] = (r == c) ? 1.0 : 0.0;
    }
  // (every loop is unrolled and the pivot row is swapped in by selects, so
  // the matrix stays in registers)
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int p = c;
    double best = fabs(a[c][c]);
#pragma unroll
    for (int r = c + 1; r < 4; ++r)
      if (fabs(a[r][c]) > best) { p = r; best = fabs(a[r][c]); }
#pragma unroll
    for (int r = c + 1; r < 4; ++r) {
      const bool sw = r == p;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double x = a[c][k], y = a[r][k];
        a[c][k] = sw ? y : x;
        a[r][k] = sw ? x : y;
      }
    }
    if (a[c][c] == 0.0) return false;
    const double d = a[c][c];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[c][k] = a[c][k] / d;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      if (f == 0.0) continue;
#pragma unroll
      for (int k = 0; k < 8; ++k) a[r][k] = a[r][k] - f * a[c][k];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) inv[r * 4 + c] = a[r][c + 4];
  return true;
}

__device__ __forceinline__ void split(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

__device__ void view_params(const BcViewIn& in, BcViewParams& vp, int tile_shift) {
#pragma clang fp contract(off)
  // (ordered so that few matrices are live at once: one thread computes this,
  // and the 4x4 inverse then fits in registers)
  double PM[16], Q[16];
  bool persp;
  double e[3], dir[3];
  {
    double M[16], P[16];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        M[r * 4 + c] = in.mv[c * 4 + r];
        P[r * 4 + c] = in.pr[c * 4 + r];
      }
    mat4_mul(P, M, PM);
    persp = (P[12] == 0.0 && P[13] == 0.0 && P[14] == -1.0 && P[15] == 0.0);
    // eye e_a = -((R0a t0 + R1a t1) + R2a t2), without fused multiply-add
    for (int a = 0; a < 3; ++a) {
      e[a] = -((M[0 * 4 + a] * M[3] + M[1 * 4 + a] * M[7]) + M[2 * 4 + a] * M[11]);
      dir[a] = -M[2 * 4 + a];
    }
  }
  for (int k = 0; k < 16; ++k) vp.pm[k] = PM[k];
  mat4_inv(PM, Q);
  vp.kind = persp ? 0 : 1;
  vp.width = in.width;
  vp.height = in.height;
  vp.tile_shift = tile_shift;
  vp.tiles_x = (in.width + (1 << tile_shift) - 1) >> tile_shift;
  vp.tiles_y = (in.height + (64 >> tile_shift) - 1) >> (6 - tile_shift);
  split(in.step, vp.dt_hi, vp.dt_lo);
  split(1.0 / in.step, vp.idt_hi, vp.idt_lo);
  split(1.0 / (double)in.width, vp.iw_hi, vp.iw_lo);
  split(1.0 / (double)in.height, vp.ih_hi, vp.ih_lo);
  vp.tau = (float)in.tau;
  for (int a = 0; a < 3; ++a) {
    vp.eye[a] = e[a];
    vp.dir[a] = dir[a];
  }
  double E[3], A[3], B[3], C[3];
  if (persp) {
    // far point w(x, y) = Q (x, y, 1, 1); direction of dehom(w) - e is w.xyz - e w.w
    double sgn = 1.0;
    const double w00 = -Q[12] - Q[13] + Q[14] + Q[15];
    if (w00 < 0.0) sgn = -1.0;
    for (int a = 0; a < 3; ++a) {
      E[a] = e[a];
      A[a] = sgn * (Q[a * 4 + 0] - e[a] * Q[12]);
      B[a] = sgn * (Q[a * 4 + 1] - e[a] * Q[13]);
      C[a] = sgn * ((Q[a * 4 + 2] + Q[a * 4 + 3]) - e[a] * (Q[14] + Q[15]));
    }
  } else {
    // origin on the near plane o(x, y) = Q (x, y, -1, 1); direction Q (0, 0, 2, 0)
    double n = 0.0;
    for (int a = 0; a < 3; ++a) n = n + Q[a * 4 + 2] * Q[a * 4 + 2];
    n = sqrt(n);
    for (int a = 0; a < 3; ++a) {
      E[a] = Q[a * 4 + 3] - Q[a * 4 + 2];
      A[a] = Q[a * 4 + 0];
      B[a] = Q[a * 4 + 1];
      C[a] = Q[a * 4 + 2] / n;
    }
  }
  for (int a = 0; a < 3; ++a) {
    split(E[a], vp.e_hi[a], vp.e_lo[a]);
    split(A[a], vp.a_hi[a], vp.a_lo[a]);
    split(B[a], vp.b_hi[a], vp.b_lo[a]);
    split(C[a], vp.c_hi[a], vp.c_lo[a]);
  }
}

// visibility key: power distance from the eye (perspective) or the centre's
// projection on the view direction (orthographic), FP64 left to right, no FMA
__device__ double brick_key(const BcViewParams& vp, const BcBrick& b) {
#pragma clang fp contract(off)
  double k = 0.0;
  if (vp.kind == 0) {
    for (int a = 0; a < 3; ++a) {
      const double p = (vp.eye[a] - (double)b.lo[a]) * (vp.eye[a] - (double)b.hi[a]);
      k = k + p;
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      const double c = ((double)b.lo[a] + (double)b.hi[a]) / 2.0;
      k = k + c * vp.dir[a];
    }
  }
  return k;
}

// conservative rendering rectangle in whole tiles: bounding box of the eight
// projected corners widened by one pixel; the whole frame when a corner lies
// behind the eye or the eye is inside the brick
__device__ void brick_rect(const BcViewParams& vp, const BcBrick& b, int32_t* r) {
#pragma clang fp contract(off)
  const int W = vp.width, H = vp.height;
  bool full = false;
  if (vp.kind == 0) {
    bool inside = true;
    for (int a = 0; a < 3; ++a) inside = inside && vp.eye[a] >= b.lo[a] && vp.eye[a] <= b.hi[a];
    full = inside;
  }
  double xmin = DBL_MAX, xmax = -DBL_MAX, ymin = DBL_MAX, ymax = -DBL_MAX;
  for (int c = 0; c < 8 && !full; ++c) {
    const double X = (c & 1) ? b.hi[0] : b.lo[0];
    const double Y = (c & 2) ? b.hi[1] : b.lo[1];
    const double Z = (c & 4) ? b.hi[2] : b.lo[2];
    double clip[4];
    for (int i = 0; i < 4; ++i)
      clip[i] = ((vp.pm[i * 4 + 0] * X + vp.pm[i * 4 + 1] * Y) + vp.pm[i * 4 + 2] * Z) + vp.pm[i * 4 + 3];
    if (!(clip[3] > 0.0)) { full = true; break; }
    const double px = (clip[0] / clip[3] + 1.0) * (0.5 * W) - 0.5;
    const double py = (1.0 - clip[1] / clip[3]) * (0.5 * H) - 0.5;
    xmin = fmin(xmin, px); xmax = fmax(xmax, px);
    ymin = fmin(ymin, py); ymax = fmax(ymax, py);
  }
  int x0, x1, y0, y1;   // inclusive pixel bounds
  if (full) {
    x0 = 0; y0 = 0; x1 = W - 1; y1 = H - 1;
  } else {
    if (xmax < -1.0 || ymax < -1.0 || xmin > W || ymin > H) {
      r[0] = r[1] = r[2] = r[3] = 0;
      return;
    }
    x0 = (int)fmax(floor(xmin) - 1.0, 0.0);
    y0 = (int)fmax(floor(ymin) - 1.0, 0.0);
    x1 = (int)fmin(ceil(xmax) + 1.0, (double)(W - 1));
    y1 = (int)fmin(ceil(ymax) + 1.0, (double)(H - 1));
    if (x1 < x0 || y1 < y0) {
      r[0] = r[1] = r[2] = r[3] = 0;
      return;
    }
  }
  const int sx = vp.tile_shift, sy = 6 - vp.tile_shift;
  r[0] = x0 >> sx;
  r[1] = y0 >> sy;
  r[2] = (x1 >> sx) + 1;
  r[3] = (y1 >> sy) + 1;
}

// brick counts up to which the visibility order is a rank count rather than
// a bitonic network (nb^2 / 1024 comparisons per thread against log^2 nb
// barriers)
constexpr int kRankSortMax = 256;

__global__ __launch_bounds__(1024) void setup_kernel(BcFramePtrs f) {
  __shared__ double skey[BC_MAX_BRICKS];
  __shared__ int32_t sidx[BC_MAX_BRICKS];
  __shared__ int32_t spart[1024 + 1];
  const int tid = threadIdx.x;
  const int nv = f.n_views;
  const int nb = f.n_bricks;
  // the pass inputs, read straight from the host's pinned buffer (two words
  // per thread for a 256-entry table) instead of a separate copy ahead of the
  // kernel; no thread has read `fin` before the barrier
  if (f.fin_src) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(f.fin_src);
    uint32_t* dst = reinterpret_cast<uint32_t*>(const_cast<BcFrameIn*>(f.fin));
    for (int i = tid; i < f.fin_bytes / 4; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
  }
  // a conditional pass without the fall-back flag has no work: only its
  // (empty) work list below is written
  const bool skip = f.fin->conditional && !f.ctr->fallback;
  if (tid < nv && !skip) view_params(f.fin->views[tid], f.views[tid], f.tile_shift);
  __syncthreads();
  int np2 = 1;
  while (np2 < nb) np2 <<= 1;
  // views whose padded key arrays fit side by side are ordered concurrently,
  // each by its own group of threads; the groups pass the same barriers, as
  // every view has the same brick count
  const int groups = (nv > 1 && nv * np2 <= BC_MAX_BRICKS) ? nv : 1;
  const int T = (int)blockDim.x / groups;
  const int grp = min(tid / T, groups - 1), t = tid - grp * T;
  const bool member = tid < groups * T;
  double* gkey = skey + grp * np2;
  int32_t* gidx = sidx + grp * np2;
  for (int v0 = 0; v0 < (skip ? 0 : nv); v0 += groups) {
    const int v = v0 + grp;
    const bool on = member && v < nv;
    const BcViewParams& vp = f.views[on ? v : v0];
    if (on) {
      for (int i = t; i < np2; i += T) {
        if (i < nb) {
          gkey[i] = brick_key(vp, f.bricks[i]);
          gidx[i] = i;
        } else {
          gkey[i] = DBL_MAX;
          gidx[i] = 0x7fffffff;
        }
      }
    }
    __syncthreads();
    if (nb <= kRankSortMax) {
      // few bricks: each thread counts the (key, index) pairs below its own
      // (one pass, one barrier; the same order as the network below); a
      // group has at least 256 threads
      int rank = 0;
      if (on && t < nb) {
        const double k = gkey[t];
        for (int j = 0; j < nb; ++j) {
          const double kj = gkey[j];
          rank += (kj < k || (kj == k && j < t)) ? 1 : 0;
        }
      }
      __syncthreads();
      if (on && t < nb) gidx[rank] = t;
      __syncthreads();
    } else {
      for (int k = 2; k <= np2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          if (on) {
            for (int i = t; i < np2; i += T) {
              const int ixj = i ^ j;
              if (ixj > i) {
                const bool up = (i & k) == 0;
                const double ka = gkey[i], kb = gkey[ixj];
                const int ia = gidx[i], ib = gidx[ixj];
                const bool gt = (ka > kb) || (ka == kb && ia > ib);
                if (gt == up) {
                  gkey[i] = kb; gkey[ixj] = ka;
                  gidx[i] = ib; gidx[ixj] = ia;
                }
              }
            }
          }
          __syncthreads();
        }
      }
    }
    if (on) {
      for (int i = t; i < nb; i += T) f.order[v * nb + i] = gidx[i];
      for (int b = t; b < nb; b += T) brick_rect(vp, f.bricks[b], f.rects + ((int64_t)v * nb + b) * 4);
    }
    __syncthreads();
  }
  // work items: entry (b, v) owns the selected tiles of its rectangle (none in
  // a conditional pass without the fall-back flag).  Entries are numbered in
  // queue order -- bricks grouped by b % Q -- so that queue q (served first by
  // the waves of XCD q) holds whole bricks and the XCDs' L2 caches hold
  // different bricks.
  const int ts = f.fin->tile_stride, tox = f.fin->tile_ox, toy = f.fin->tile_oy;
  const int Q = f.n_queues;
  const int K = nb * nv;
  const int seg = (K + blockDim.x - 1) / blockDim.x;
  const int k0 = tid * seg, k1 = min(k0 + seg, K);
  auto count_at = [&](int pos) -> int32_t {
    int b, v;
    queue_entry(pos, nb, nv, Q, b, v);
    const int32_t* r = f.rects + ((int64_t)v * nb + b) * 4;
    return skip ? 0 : sel_count(r[0], r[2], ts, tox) * sel_count(r[1], r[3], ts, toy);
  };
  int32_t sum = 0;
  for (int k = k0; k < k1; ++k) sum += count_at(k);
  // exclusive scan of the threads' sums: within each wave by shuffles, then
  // over the waves' totals
  {
    const int lane = tid & 63, wave = tid >> 6;
    int32_t x = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) spart[wave] = x;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < wave; ++w) before += spart[w];
    __syncthreads();
    spart[tid] = before + x - sum;
    if (tid == (int)blockDim.x - 1) spart[blockDim.x] = before + x;
  }
  __syncthreads();
  if (tid == 0) {
    const int32_t run = spart[blockDim.x];
    f.item_perm[K] = run;
    f.item_base[K] = run;
    const uint32_t n_items = (uint32_t)min((int64_t)run, f.max_items);
    f.ctr->n_items = n_items;
    if (f.fin->reset_counters) {
      f.ctr->nominal = 0ull;
      f.ctr->evaluated = 0ull;
      f.ctr->total_items = n_items;
    } else {
      f.ctr->total_items += n_items;
    }
  }
  __syncthreads();
  int32_t run = spart[tid];
  for (int k = k0; k < k1; ++k) {
    f.item_perm[k] = run;
    int b, v;
    queue_entry(k, nb, nv, Q, b, v);
    f.item_base[b * nv + v] = run;
    const int32_t* r = f.rects + ((int64_t)v * nb + b) * 4;
    f.item_entry[k] = make_int4(b | (v << 16), sel_count(r[0], r[2], ts, tox), sel_first(r[0], ts, tox),
                                sel_first(r[1], ts, toy));
    run += count_at(k);
  }
  __syncthreads();
  if (tid < 8) {
    f.ctr->q[tid].next = 0u;
    int g0 = 0;
    for (int g = 0; g < min(tid, Q); ++g) g0 += group_size(nb, Q, g);
    f.ctr->qbound[tid] = tid < Q ? (uint32_t)f.item_perm[g0 * nv] : (uint32_t)f.item_perm[K];
  }
  if (tid == 8) {
    f.ctr->qbound[8] = (uint32_t)f.item_perm[K];
    f.ctr->n_queues = (uint32_t)Q;
  }
}

// One workgroup per 4x4 block of screen tiles (16 waves, one tile each).  The
// workgroup first culls the view's visibility order down to the bricks whose
// rectangle meets the block (order kept, in LDS), so each wave folds only the
// sub-images that can cover its tile.
constexpr int kCompBlock = 4;
__global__ __launch_bounds__(1024) void composite_kernel(BcFramePtrs f, float4* __restrict__ out) {
  __shared__ int32_t list[BC_MAX_BRICKS];
  __shared__ int32_t wave_count[16];
  __shared__ int32_t n_list;
  if (f.fin->conditional && !f.ctr->fallback) return;
  const int v = blockIdx.z;
  const int nb = f.n_bricks, nv = f.n_views;
  const int W = f.width, H = f.height;
  const int ts = f.fin->tile_stride, tox = f.fin->tile_ox, toy = f.fin->tile_oy;
  const int bx0 = blockIdx.x * kCompBlock, by0 = blockIdx.y * kCompBlock;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ordered compaction of the bricks whose rectangle meets this block of tiles
  if (tid == 0) n_list = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int k = base + tid;
    bool keep = false;
    int b = 0;
    if (k < nb) {
      b = f.order[v * nb + k];
      const int32_t* r = f.rects + ((int64_t)v * nb + b) * 4;
      keep = r[0] < bx0 + kCompBlock && r[2] > bx0 && r[1] < by0 + kCompBlock && r[3] > by0;
    }
    const uint64_t bal = __ballot(keep);
    if (lane == 0) wave_count[wave] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wave_count[w];
    if (keep) list[n_list + before + __popcll(bal & ((1ull << lane) - 1ull))] = b;
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int w = 0; w < 16; ++w) t += wave_count[w];
      n_list += t;
    }
    __syncthreads();
  }
  const int tx = bx0 + (wave % kCompBlock), ty = by0 + (wave / kCompBlock);
  const int tsh = f.tile_shift, tw = 1 << tsh, th = 64 >> tsh;
  const int tiles_x = (W + tw - 1) >> tsh, tiles_y = (H + th - 1) >> (6 - tsh);
  if (tx >= tiles_x || ty >= tiles_y) return;
  if (tx % ts != tox || ty % ts != toy) return;
  const int px = tx * tw + (lane & (tw - 1));
  const int py = ty * th + (lane >> tsh);
  float4 F = make_float4(0.f, 0.f, 0.f, 0.f);
  float M = -INFINITY;
  const int n = n_list;
  // the list in groups of 64 entries: lane j finds the sub-image tile of
  // entry j for this wave's screen tile (-1: its rectangle misses the tile),
  // all lanes' loads in flight together; then the wave folds the tiles in
  // list order, four sub-image loads in flight
  for (int base = 0; base < n; base += 64) {
    const int m = min(64, n - base);
    int my_item = -1;
    if (lane < m) {
      const int b = list[base + lane];
      const int32_t* r = f.rects + ((int64_t)v * nb + b) * 4;
      const int r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
      if (tx >= r0 && tx < r2 && ty >= r1 && ty < r3) {
        const int fx = sel_first(r0, ts, tox), fy = sel_first(r1, ts, toy);
        const int cx = sel_count(r0, r2, ts, tox);
        const int64_t item = (int64_t)f.item_base[b * nv + v] + (int64_t)((ty - fy) / ts) * cx + (tx - fx) / ts;
        if (item < (int64_t)f.max_items) my_item = (int)item;
      }
    }
    for (int k0 = 0; k0 < m; k0 += 4) {
      int it[4];
      float4 S[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) it[u] = k0 + u < m ? __shfl(my_item, k0 + u) : -1;
      if (f.op == 1) {
        const float* subf = reinterpret_cast<const float*>(f.sub);
        float m4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) m4[u] = it[u] >= 0 ? subf[(int64_t)it[u] * 64 + lane] : -INFINITY;
#pragma unroll
        for (int u = 0; u < 4; ++u) M = fmaxf(M, m4[u]);
        continue;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        S[u] = it[u] >= 0 ? f.sub[(int64_t)it[u] * 64 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float om = 1.0f - F.w;
        F.x = __builtin_fmaf(om, S[u].x, F.x);
        F.y = __builtin_fmaf(om, S[u].y, F.y);
        F.z = __builtin_fmaf(om, S[u].z, F.z);
        F.w = __builtin_fmaf(om, S[u].w, F.w);
      }
    }
  }
  if (f.op == 1 && M != -INFINITY) {
    // maximum intensity projection: the largest brick maximum (any order),
    // then the colour map; no sample anywhere leaves the pixel clear
    const int K = f.fin->K;
    const float4* tab = reinterpret_cast<const float4*>(f.fin->table);
    float x = __builtin_fmaf(M, f.fin->tf_scale, f.fin->tf_bias);
    x = fminf(fmaxf(x, 0.0f), (float)(K - 1));
    const int i = min((int)x, K - 2);
    const float t = x - (float)i;
    const float4 a = tab[i], b = tab[i + 1];
    F = make_float4(__builtin_fmaf(t, b.x - a.x, a.x), __builtin_fmaf(t, b.y - a.y, a.y),
                    __builtin_fmaf(t, b.z - a.z, a.z), __builtin_fmaf(t, b.w - a.w, a.w));
  }
  if (px < W && py < H) out[((int64_t)v * H + py) * W + px] = F;
}

// Few bricks (up to kTileCompMax): one wave per screen tile, four per
// workgroup (a 2x2 block of tiles), no culling pass and no barrier.  Lane j
// takes entries j, j + 64, ... of the view's visibility order and finds the
// brick's sub-image tile for this screen tile (its rectangle, and the brick's
// first work item, loaded together); the wave then folds the covering tiles
// in visibility order, four sub-image loads in flight.  Entries that do not
// cover the tile fold as zero in composite_kernel, which changes no bit, so
// the two kernels' images are identical.
constexpr int kTileCompMax = 128;
__global__ __launch_bounds__(256) void composite_tile_kernel(BcFramePtrs f, float4* __restrict__ out) {
  if (f.fin->conditional && !f.ctr->fallback) return;
  const int v = blockIdx.z;
  const int nb = f.n_bricks, nv = f.n_views;
  const int W = f.width, H = f.height;
  const int ts = f.fin->tile_stride, tox = f.fin->tile_ox, toy = f.fin->tile_oy;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tx = (int)blockIdx.x * 2 + (wave & 1), ty = (int)blockIdx.y * 2 + (wave >> 1);
  const int tsh = f.tile_shift, tw = 1 << tsh, th = 64 >> tsh;
  const int tiles_x = (W + tw - 1) >> tsh, tiles_y = (H + th - 1) >> (6 - tsh);
  if (tx >= tiles_x || ty >= tiles_y) return;
  if (tx % ts != tox || ty % ts != toy) return;
  const int px = tx * tw + (lane & (tw - 1));
  const int py = ty * th + (lane >> tsh);
  float4 F = make_float4(0.f, 0.f, 0.f, 0.f);
  float M = -INFINITY;
  for (int base = 0; base < nb; base += 64) {
    const int k = base + lane;
    int my_item = -1;
    if (k < nb) {
      const int b = f.order[v * nb + k];
      const int32_t* r = f.rects + ((int64_t)v * nb + b) * 4;
      const int r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
      const int64_t first = f.item_base[b * nv + v];
      if (tx >= r0 && tx < r2 && ty >= r1 && ty < r3) {
        const int fx = sel_first(r0, ts, tox), fy = sel_first(r1, ts, toy);
        const int cx = sel_count(r0, r2, ts, tox);
        const int64_t item = first + (int64_t)((ty - fy) / ts) * cx + (tx - fx) / ts;
        if (item < (int64_t)f.max_items) my_item = (int)item;
      }
    }
    uint64_t cover = __ballot(my_item >= 0);
    while (cover) {
      int it[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        it[u] = -1;
        if (cover) {
          const int j = __builtin_ctzll(cover);
          cover &= cover - 1ull;
          it[u] = __shfl(my_item, j);
        }
      }
      if (f.op == 1) {
        const float* subf = reinterpret_cast<const float*>(f.sub);
        float m4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) m4[u] = it[u] >= 0 ? subf[(int64_t)it[u] * 64 + lane] : -INFINITY;
#pragma unroll
        for (int u = 0; u < 4; ++u) M = fmaxf(M, m4[u]);
        continue;
      }
      float4 S[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        S[u] = it[u] >= 0 ? f.sub[(int64_t)it[u] * 64 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float om = 1.0f - F.w;
        F.x = __builtin_fmaf(om, S[u].x, F.x);
        F.y = __builtin_fmaf(om, S[u].y, F.y);
        F.z = __builtin_fmaf(om, S[u].z, F.z);
        F.w = __builtin_fmaf(om, S[u].w, F.w);
      }
    }
  }
  if (f.op == 1 && M != -INFINITY) {
    const int K = f.fin->K;
    const float4* tab = reinterpret_cast<const float4*>(f.fin->table);
    float x = __builtin_fmaf(M, f.fin->tf_scale, f.fin->tf_bias);
    x = fminf(fmaxf(x, 0.0f), (float)(K - 1));
    const int i = min((int)x, K - 2);
    const float t = x - (float)i;
    const float4 a = tab[i], b = tab[i + 1];
    F = make_float4(__builtin_fmaf(t, b.x - a.x, a.x), __builtin_fmaf(t, b.y - a.y, a.y),
                    __builtin_fmaf(t, b.z - a.z, a.z), __builtin_fmaf(t, b.w - a.w, a.w));
  }
  if (px < W && py < H) out[((int64_t)v * H + py) * W + px] = F;
}

// Learned frame: PSNR (peak 1) of the upsampled image against the plain
// render over the validation tiles, and the fall-back decision.
__global__ __launch_bounds__(1024) void psnr_kernel(BcFramePtrs f, const float4* __restrict__ ref,
                                                    const float4* __restrict__ img) {
  // FP32 throughout: each thread keeps a compensated (Kahan) sum of its
  // pixels' squared differences, and the block adds the 1024 partial sums
  // pairwise (relative error about 10 roundings)
  __shared__ float red[1024];
  __shared__ int nred[1024];
  const int ts = f.fin->tile_stride, tox = f.fin->tile_ox, toy = f.fin->tile_oy;
  const int W = f.width, H = f.height, nv = f.n_views;
  const int tsh = f.tile_shift, tw = 1 << tsh, th = 64 >> tsh;
  const int tiles_x = (W + tw - 1) >> tsh, tiles_y = (H + th - 1) >> (6 - tsh);
  const int sx = sel_count(0, tiles_x, ts, tox), sy = sel_count(0, tiles_y, ts, toy);
  const int fx = sel_first(0, ts, tox), fy = sel_first(0, ts, toy);
  const int64_t total = (int64_t)nv * sx * sy * 64;
  float acc = 0.0f, comp = 0.0f;
  int cnt = 0;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int lane = (int)(e & 63);
    const int64_t t = e >> 6;
    const int v = (int)(t / ((int64_t)sx * sy));
    const int rem = (int)(t % ((int64_t)sx * sy));
    const int tx = fx + (rem % sx) * ts, ty = fy + (rem / sx) * ts;
    const int px = tx * tw + (lane & (tw - 1)), py = ty * th + (lane >> tsh);
    if (px >= W || py >= H) continue;
    const int64_t i = ((int64_t)v * H + py) * W + px;
    const float4 a = ref[i], b = img[i];
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
    const float term = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, dw * dw)));
    const float y = term - comp;
    const float t2 = acc + y;
    comp = (t2 - acc) - y;
    acc = t2;
    cnt += 4;
  }
  red[threadIdx.x] = acc;
  nred[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      nred[threadIdx.x] += nred[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float mse = nred[0] > 0 ? red[0] / (float)nred[0] : 0.0f;
    const float p = mse > 0.0f ? 10.0f * log10f(1.0f / mse) : INFINITY;
    f.ctr->psnr_db = p;
    f.ctr->fallback = (p < f.fin->psnr_threshold) ? 1u : 0u;
  }
}

}  // namespace

hipError_t bc_launch_setup(const BcFramePtrs& f, hipStream_t st) {
  setup_kernel<<<1, 1024, 0, st>>>(f);
  return hipGetLastError();
}

hipError_t bc_launch_psnr(const BcFramePtrs& f, const float4* ref, const float4* img, hipStream_t st) {
  psnr_kernel<<<1, 1024, 0, st>>>(f, ref, img);
  return hipGetLastError();
}

hipError_t bc_launch_composite(const BcFramePtrs& f, float4* out, hipStream_t st) {
  const int tsh = f.tile_shift;
  const int tiles_x = (f.width + (1 << tsh) - 1) >> tsh, tiles_y = (f.height + (64 >> tsh) - 1) >> (6 - tsh);
  if (f.n_bricks <= kTileCompMax) {
    dim3 grid((tiles_x + 1) / 2, (tiles_y + 1) / 2, f.n_views);
    composite_tile_kernel<<<grid, 256, 0, st>>>(f, out);
  } else {
    dim3 grid((tiles_x + kCompBlock - 1) / kCompBlock, (tiles_y + kCompBlock - 1) / kCompBlock, f.n_views);
    composite_kernel<<<grid, 1024, 0, st>>>(f, out);
  }
  return hipGetLastError();
}
