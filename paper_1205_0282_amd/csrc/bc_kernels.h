// Kernel launchers called by the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "bc_types.h"

struct BcLoadSrc {
  const void* ptr;        // device pointer
  int64_t strides[3];     // elements (x, y, z)
  int32_t origin[3];      // global voxel coordinates of element [0][0][0]
  int32_t dims[3];        // global cube dims
  int32_t dtype;          // 0 float32, 1 float16
};

hipError_t bc_launch_init_minmax(BcCounters* ctr, int n, hipStream_t st);
// bricks [first, first + count): max_rows bounds each brick's ghosted rows
// (y * z extent); the encode's max_rows bounds its rows of micro-blocks along x
// (y * z extent in micro-blocks)
hipError_t bc_launch_minmax(const BcLoadSrc& src, const BcBrick* bricks, int first, int count, int max_rows,
                            BcCounters* ctr, hipStream_t st);
hipError_t bc_launch_finalize(BcBrick* bricks, const BcCounters* ctr, int first, int count, int storage,
                              hipStream_t st);
hipError_t bc_launch_encode(const BcLoadSrc& src, const BcBrick* bricks, int first, int count, int64_t max_rows,
                            int storage, void* pool, hipStream_t st);

struct BcFramePtrs {
  const BcFrameIn* fin;
  BcViewParams* views;
  const BcBrick* bricks;
  int32_t* order;         // [BC_MAX_VIEWS][n_bricks]
  int32_t* rects;         // [BC_MAX_VIEWS][n_bricks][4] tiles (x0, y0, x1, y1)
  int32_t* item_base;     // [n_bricks * n_views + 1] first item of entry b * n_views + v
  int32_t* item_perm;     // [n_bricks * n_views + 1] first item of the entry at each queue-order position
  int4* item_entry;       // [n_bricks * n_views] the entry at each queue-order position: brick | view << 16,
                          // its selected tile columns, its first selected tile x and y
  BcCounters* ctr;
  float4* sub;            // sub-image tiles: [max_items][64] (one float per ray, read as
                          // float[max_items][64], for maximum intensity projection)
  const void* pool;
  uint32_t* occ;          // cell-occupancy bits of every brick
  int32_t ess;            // skip samples in clear cells
  int32_t chunk;          // samples per occupancy-mask chunk of the ray caster (32 or 64)
  int32_t n_queues;       // 8: bricks split over one work queue per XCD; 1: one queue
  int32_t K;              // transfer-function entries
  int32_t op;             // 0 front-to-back compositing, 1 maximum intensity projection
  int32_t step_policy;    // 0 the view's fixed step, 1 one sample per voxel slice
  int32_t n_bricks, n_views;
  int32_t gdims[3];
  int64_t max_items;
  int32_t storage;
  int32_t width, height;  // frame size (all views share it)
  int32_t urgent;         // 1: the ray caster's waves issue at raised priority (2, and 3 while
                          // evaluating); 0: at the base levels (0 and 1), for a pass that runs
                          // beside a more urgent one
  int32_t tile_shift;     // screen tiles are (1 << tile_shift) x (64 >> tile_shift) pixels
  // the pass inputs in host-coherent pinned memory, which the set-up kernel
  // copies to `fin` before it reads them (nullptr: `fin` already holds them)
  const BcFrameIn* fin_src;
  int32_t fin_bytes;      // bytes of the pass inputs to copy (a multiple of 4)
};

hipError_t bc_launch_setup(const BcFramePtrs& f, hipStream_t st);
hipError_t bc_launch_classify(const BcFramePtrs& f, int max_words, hipStream_t st);
hipError_t bc_launch_render(const BcFramePtrs& f, int n_workgroups, hipStream_t st);
hipError_t bc_launch_composite(const BcFramePtrs& f, float4* out, hipStream_t st);
hipError_t bc_launch_psnr(const BcFramePtrs& f, const float4* ref, const float4* img, hipStream_t st);

// Queue order of the (brick, view) entries: bricks grouped by b % Q, then b,
// then view.  Returns the position of entry (b, v) and, inversely, the entry at
// a position.
__device__ __forceinline__ int group_size(int nb, int Q, int x) { return x < nb ? (nb - x + Q - 1) / Q : 0; }
__device__ __forceinline__ int queue_pos(int b, int v, int nb, int nv, int Q) {
  const int x = b % Q;
  int before = 0;
  for (int g = 0; g < x; ++g) before += group_size(nb, Q, g);
  return (before + b / Q) * nv + v;
}
__device__ __forceinline__ void queue_entry(int pos, int nb, int nv, int Q, int& b, int& v) {
  const int e = pos / nv;
  v = pos % nv;
  int cum = 0, x = 0;
  for (; x < Q - 1; ++x) {
    const int g = group_size(nb, Q, x);
    if (e < cum + g) break;
    cum += g;
  }
  b = x + (e - cum) * Q;
}

// tile selection {t : t % s == o}: first selected tile >= lo, count in [lo, hi)
__device__ __forceinline__ int sel_first(int lo, int s, int o) { return lo + ((o - lo) % s + s) % s; }
__device__ __forceinline__ int sel_count(int lo, int hi, int s, int o) {
  const int f = sel_first(lo, s, o);
  return f < hi ? (hi - 1 - f) / s + 1 : 0;
}
