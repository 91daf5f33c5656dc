// Layouts shared by the host runtime and the kernels of the bricked ray caster.
#pragma once
#include <stddef.h>
#include <stdint.h>

#define BC_MAX_VIEWS 4
#define BC_MAX_BRICKS 4096
#define BC_MAX_K 4096
#define BC_TILE 8          // default screen tile edge (pixels): one wave of 64 rays per work item;
                           // tiles may also be 16 x 4 or 4 x 16 (always 64 pixels)
#define BC_MB 4            // micro-block edge (voxels)
// A 4 x 4 x 4 micro-block is stored as 16 rows (y, z) of 5 elements: voxels
// x = 0..3 of the row and, fifth, the first voxel of the next micro-block along
// x, so the +x neighbour of every voxel is the next element (one paired load).
#define BC_ROW 5
#define BC_MB_ELEMS 80
#define BC_TF_LDS 1024     // transfer functions up to this many entries are staged in LDS

// A rendering request as the viewer sends it (FP64, OpenGL column-major).
struct BcViewIn {
  double mv[16];
  double pr[16];
  int32_t width, height;
  double step, tau;
};

// Per-pass input copied host -> device before the frame.  A plain frame is one
// pass; a learned frame is three (coarse render, sparse validation render,
// conditional full render).
struct BcFrameIn {
  BcViewIn views[BC_MAX_VIEWS];
  int32_t n_views, K;
  float tf_scale, tf_bias;   // table coordinate x = v * tf_scale + tf_bias
  int32_t tile_stride;       // 1: every screen tile; s > 1: tiles with tx % s == ox and ty % s == oy
  int32_t tile_ox, tile_oy;
  int32_t reset_counters;    // the pass starts the frame's sample counters
  int32_t conditional;       // the pass runs only if the validation set the fall-back flag
  float psnr_threshold;      // validation pass: dB below which the frame falls back
  int32_t op;                // 0 front-to-back compositing, 1 maximum intensity projection
  int32_t step_policy;       // 0 the view's fixed step, 1 one sample per voxel slice (per ray)
  // compositing: opacity-corrected premultiplied RGBA entries; maximum
  // intensity projection: the straight colour-map entries (only K used)
  float table[BC_MAX_K][4];
};

// Derived per-view quantities written by the FP64 setup kernel.  Vectors used
// per ray are stored as double-float pairs (hi + lo) so that FP32 arithmetic
// can place samples as accurately as FP64 would.
struct BcViewParams {
  int32_t kind;              // 0 perspective, 1 orthographic
  int32_t width, height, tiles_x, tiles_y;
  int32_t tile_shift;        // log2 of the screen tile width: tiles are (1 << s) x (64 >> s) pixels
  float dt_hi, dt_lo;        // step (double-float)
  float idt_hi, idt_lo;      // 1 / step
  float iw_hi, iw_lo;        // 1 / width
  float ih_hi, ih_lo;        // 1 / height
  float tau;
  float pad1;
  // perspective: e = eye, a/b/c: unnormalised direction u(x, y) = a x + b y + c
  // orthographic: e = origin at NDC (0, 0) on the near plane, a/b its NDC
  // derivatives, c = unit view direction
  float e_hi[3], e_lo[3];
  float a_hi[3], a_lo[3];
  float b_hi[3], b_lo[3];
  float c_hi[3], c_lo[3];
  double eye[3];
  double dir[3];
  double pm[16];             // P*M, row-major
};

struct BcBrick {
  int32_t lo[3], hi[3];      // core box, global voxel coordinates
  int32_t gdim[3];           // stored dims: core + 2 ghosts, padded to a multiple of 4
  int32_t mb[3];             // micro-blocks per axis (BC_MB_ELEMS elements each)
  int64_t offset;            // first element of the brick in the pool
  int64_t occ_offset;        // first 32-bit word of the brick's cell-occupancy bits
  int32_t occ_w[3];          // occupancy words per axis (one word = 4 x 4 x 2 cells)
  int32_t pad_;
  float scale, offs;         // decode v = q * scale + offs (FP8); 1, 0 otherwise
  float vmin, vmax;          // range of the source (core + ghost) values
  float dmax;                // largest value the stored elements decode to
  int32_t pad2_;
};

// Device counters.  The cache lines that the ray-casting waves update with
// atomics (one per work queue, one for the sample counts) hold nothing else,
// so the read-only fields the waves load are never in a line under atomic
// traffic.
struct BcQueueCounter {
  uint32_t next;             // next item of the queue (relative to its start)
  uint32_t pad_[31];
};
struct BcCounters {
  // written by the set-up kernel, read-only during ray casting
  uint32_t n_items;          // work items of the pass
  uint32_t n_queues;         // work queues of the pass (one per XCD, or one)
  uint32_t qbound[9];        // queue q holds items [qbound[q], qbound[q+1])
  uint32_t fallback;         // learned frame: validation PSNR below threshold
  float psnr_db;             // learned frame: PSNR of the validation tiles
  uint32_t total_items;      // work items of all passes of the frame
  uint32_t pad0_[18];
  // sample counts, added once per wave at its end
  unsigned long long nominal;
  unsigned long long evaluated;
  uint32_t pad1_[28];
  BcQueueCounter q[8];
  uint32_t minmax[BC_MAX_BRICKS][2];   // load time: ordered-int min/max per brick
};

static_assert(offsetof(BcCounters, nominal) == 128, "sample counts start a cache line");
static_assert(offsetof(BcCounters, q) == 256, "queue counters start a cache line");
static_assert(sizeof(BcQueueCounter) == 128, "one queue counter per cache line");
