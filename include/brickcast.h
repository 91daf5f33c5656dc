/*
 * brickcast.h -- C ABI of the bricked volume ray caster for one MI355X (gfx950).
 *
 * The calls follow the duties the paper gives each GPU's rendering thread
 * (Section 2.2, item 5): load the data into GPU memory, take a rendering
 * request made of the output frame size and the viewer's OpenGL projection
 * and transformation matrices (Section 2.3.2), work out the rendering
 * rectangle of the data and clip the ray casting to it (Section 2.3.2,
 * Figure 4), ray cast, and hand the result over for compositing
 * (Section 2.3.3).  Here one GPU holds a share of the cube split into bricks;
 * each brick is ray cast into its own sub-image and the sub-images are
 * composited front to back in visibility order.
 *
 * Conventions
 *  - Every call returns an int32 status: BC_OK (0) or a negative BC_E_* code.
 *    Nothing throws.  bc_last_error() gives the message of the last failure.
 *  - Memory: the library never allocates device memory.  bc_plan() reports
 *    the sizes of four device regions; the caller allocates them (PyTorch in
 *    the Python binding) and passes them to bc_bind_memory().  The caller owns
 *    them and must keep them alive until bc_destroy().  The library owns only
 *    small host-side state (and a small pinned host buffer for per-frame
 *    parameters).
 *  - A context is bound to one HIP device and is not thread safe: one host
 *    thread drives one context, as one CPU thread drives one GPU in the paper.
 *  - Coordinates: voxel (i, j, k) of the global cube has its centre at
 *    (i+1/2, j+1/2, k+1/2); source arrays are indexed data[z][y][x] with the
 *    strides given in elements.  Image row 0 is the top row.
 */
#ifndef BRICKCAST_H
#define BRICKCAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BC_OK = 0,
  BC_E_ARG = -1,          /* invalid argument (message says which) */
  BC_E_STATE = -2,        /* call out of order (e.g. render before load) */
  BC_E_NOMEM = -3,        /* bound memory smaller than planned, or the frame
                             needs more sub-image tiles than planned */
  BC_E_HIP = -4,          /* HIP runtime failure; message holds hipGetErrorString */
  BC_E_UNSUPPORTED = -5   /* valid but not supported by this build */
};

/* Storage form of the bricks in GPU memory. */
enum bc_format {
  BC_F32 = 0,             /* IEEE binary32 as given */
  BC_F16 = 1,             /* IEEE binary16, round to nearest even */
  BC_FP8_E4M3 = 2         /* OCP E4M3 with a per-brick scale s and offset o:
                             v = q*s + o, o = (min+max)/2, s = (max-min)/896 over
                             the brick's stored (core + ghost) values */
};

typedef struct bc_ctx bc_ctx;

/* Create a context on HIP device `hip_device` (>= 0).  hip_device = -1 makes
 * a host-only context that accepts bc_plan / bc_set_* (argument checking) but
 * refuses every call that needs a GPU with BC_E_STATE.  *out is set to NULL on
 * failure. */
int bc_create(int hip_device, bc_ctx** out);

/* Free library-owned host state.  Never frees caller memory.  NULL is a no-op. */
void bc_destroy(bc_ctx* ctx);

/* Message of the last failing call on ctx ("" if none).  Valid until the next
 * call on ctx.  ctx may be NULL (then: message of the last bc_create failure). */
const char* bc_last_error(const bc_ctx* ctx);

/* The share of the cube this GPU renders and how it is bricked (Section 2.1,
 * bricking; Section 2.3.1, the partition into sub-cubes). */
typedef struct {
  int64_t global_dims[3];   /* whole cube (x, y, z), voxels */
  int64_t share_lo[3];      /* this GPU's share, half-open box [lo, hi) */
  int64_t share_hi[3];
  int32_t brick_dims[3];    /* brick edge (e.g. 64 or 256); edge bricks are truncated */
  int32_t ghost;            /* ghost voxels per side; must be 1 */
  int32_t storage;          /* enum bc_format */
  int32_t src_dtype;        /* BC_F32 or BC_F16: element type of the source given to bc_load_bricks */
} bc_volume_desc;

/* Sizes (bytes) of the four device regions for a volume and the largest frame
 * to be rendered:
 *   bytes_out[0] brick pool     (bricks with ghosts, as 4x4x4 micro-blocks; see bc_read_brick)
 *   bytes_out[1] metadata       (brick table, views, order, rectangles, queue, counters, table,
 *                                one occupancy bit per interpolation cell of every brick)
 *   bytes_out[2] sub-images     (max_tiles sub-image tiles of 8x8 RGBA float32)
 *   bytes_out[3] load scratch   (one brick's source region, used when the source is on the host)
 * max_tiles = 0 picks a default bound: views * screen tiles * bricks when
 * that is at most 2^18 tiles, else views * screen tiles * min(bricks,
 * 2 * (bricks along x + along y + along z) + 4).  Every region is 256-byte aligned by the caller.
 * Errors: BC_E_ARG for null pointers, non-positive dims, a share outside the
 * cube, ghost != 1, unknown storage/src_dtype, max_views not in [1, 4],
 * max_w/max_h not in [1, 16384], more than 4096 bricks, a brick whose stored
 * form would take 4 GiB or more (FP32 bricks above about 940 voxels per edge). */
int bc_plan(bc_ctx* ctx, const bc_volume_desc* desc, int max_views, int max_w, int max_h,
            int64_t max_tiles, size_t bytes_out[4]);

/* Bind caller-allocated device memory (after bc_plan).  sizes[i] must be at
 * least the planned bytes_out[i] (else BC_E_NOMEM); pointers must be 256-byte
 * aligned device pointers on the context's device (else BC_E_ARG). */
int bc_bind_memory(bc_ctx* ctx, void* const dev_ptrs[4], const size_t sizes[4]);

/* Split the share into bricks with 1-voxel ghosts (clamp-replicated at the
 * cube faces), compute per-brick minimum/maximum (the paper's min/max task,
 * Section 2.3.1), encode to the storage form and lay the bricks out in GPU
 * memory.  `src` covers the share plus its ghost halo clamped to the cube, the
 * box [max(lo-1, 0), min(hi+1, N)), element type desc->src_dtype, strides in
 * elements (x, y, z).  src_on_device != 0 means `src` is a device pointer on
 * the context's device.  Synchronous: the caller may free or reuse `src` on
 * return.  Errors: BC_E_STATE before bind; BC_E_ARG for a null src or strides
 * smaller than the box rows/planes. */
int bc_load_bricks(bc_ctx* ctx, const void* src, const int64_t src_strides[3], int src_on_device);

/* Transfer function (Section 1.2: maps a voxel value to colour and opacity):
 * K straight (not premultiplied) RGBA float entries in [0, 1], entry k at
 * value vmin + k/(K-1) (vmax - vmin), opacity given per dt_ref voxels of ray
 * length.  The table is copied.  Errors (BC_E_ARG): null rgba, K not in
 * [2, 4096], vmin >= vmax or not finite, an entry outside [0, 1] or NaN,
 * dt_ref <= 0. */
int bc_set_transfer_function(bc_ctx* ctx, const float* rgba, int K, double vmin, double vmax,
                             double dt_ref);

/* One rendering request: the viewer's OpenGL matrices (column-major, as
 * glGetDoublev returns them), the frame size, the sampling step along the ray
 * in voxels and the early-ray-termination opacity (Section 2.3.2). */
typedef struct {
  double modelview[16];     /* rigid: [R t; 0 1] with R orthonormal (1e-9) */
  double projection[16];    /* perspective (row 3 = 0 0 -1 0) or orthographic (row 3 = 0 0 0 1) */
  int32_t width, height;
  double step;              /* > 0, voxels; at most 2^22 samples along the cube's diagonal */
  double ert_threshold;     /* in (0, 1]; 1 disables early termination */
} bc_view;

/* Set 1..4 views rendered together by the next frames (one launch renders all
 * of them).  All views must share width, height, step and ert_threshold, and
 * fit the planned max_views/max_w/max_h.  Copied.  Errors: BC_E_ARG for the
 * checks above (the step against the cube's diagonal once the context is
 * planned; bc_render_frame checks views set before the plan); BC_E_NOMEM if
 * the views' rendering rectangles need more sub-image tiles than planned. */
int bc_set_view(bc_ctx* ctx, const bc_view* views, int n_views);

/* Enqueue one frame on `stream` (a hipStream_t; NULL = the null stream) and
 * return.  `out`: caller-owned device buffer of n_views*height*width*4
 * float32, premultiplied RGBA (colour-mapped RGBA under BC_OP_MIP), 16-byte
 * aligned; pixels no brick covers are transparent black.  Errors (detected before anything is enqueued, `out`
 * untouched): BC_E_STATE if memory, bricks, transfer function or view is
 * missing; BC_E_ARG for a null or misaligned out, or a step (the view's, or a
 * learned frame's coarse step) that takes more than 2^22 samples along the
 * cube's diagonal. */
int bc_render_frame(bc_ctx* ctx, float* out, void* stream);

/* The same frame as bc_render_frame, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the sub-image tiles go to a fixed device array that the library
 * holds on each device it runs on (BC_STATIC_MAX_TILES tiles of 8x8 RGBA
 * float32, 64 MiB, kept until the process ends) instead of the bound
 * sub-image region, and the call allocates nothing, host or device: it
 * launches the kernels directly (it ignores BC_OPT_GRAPH, whose capture and
 * instantiation allocate) and is not counted in the bc_enable_timing window
 * (timing creates its events on demand).  Images are those of
 * bc_render_frame.  Calls on one GPU share its array and each overwrites what
 * the last left there: frames enqueued on different streams that may overlap
 * on one GPU race and give wrong images; frames on one stream, or on streams
 * that are ordered, are safe.  Errors: as bc_render_frame; BC_E_NOMEM (before
 * anything is enqueued) if the current views need more than
 * BC_STATIC_MAX_TILES sub-image tiles (the bound that bc_set_view checks
 * against the plan, here checked against the array). */
#define BC_STATIC_MAX_TILES 65536
int bc_render_frame_static(bc_ctx* ctx, float* out, void* stream);

/* Learned frames (enable = 1; needs the upsampler workspace and weights, see
 * bc_cnn_* below, and an even frame width and height).  A learned frame
 * renders the views at half the width and height with step `coarse_step`
 * (voxels; opacity corrected for that step), upsamples them with the network
 * into `out`, then renders plain (full size, the views' own step) one screen
 * tile of every validate_stride x validate_stride block of tiles (the chosen
 * tile moves from frame to frame) and compares: if the PSNR (peak 1, over the
 * RGBA of those tiles) is below psnr_threshold_db the whole frame is
 * re-rendered plain into `out` on the device, with no host round trip.  The
 * decision is in bc_get_frame_stats.  With timing enabled the three stage
 * times of a learned frame are: coarse render, network, validation plus any
 * fall-back.  Errors: BC_E_ARG for enable not 0/1, coarse_step <= 0, a
 * non-finite threshold, validate_stride outside [1, 64]. */
int bc_set_learned(bc_ctx* ctx, int enable, double coarse_step, double psnr_threshold_db, int validate_stride);

/* Ray operator and step policy of the next frames.
 *  BC_OP_COMPOSITE (default): front-to-back compositing of the transfer
 *    function's opacity-corrected premultiplied colours with early ray
 *    termination (Section 1.2); `out` holds premultiplied RGBA.
 *  BC_OP_MIP: maximum intensity projection, the operator the paper adopts
 *    (Section 2.3.3): each ray keeps the largest value it samples, a ray stops
 *    once it reaches the largest value its brick stores (the paper stops at the
 *    global maximum, Section 2.3.2; the brick's own bound gives the same
 *    image), the per-brick maxima merge in any order, and the colour map -- the
 *    transfer function's K straight entries, interpolated linearly over
 *    [vmin, vmax] and clamped, opacity and dt_ref unused -- is applied once
 *    after the merge.  A pixel whose ray takes no sample is (0, 0, 0, 0).
 *    The views' ert_threshold is not used.  Empty-space skipping stays exact:
 *    a cell is skipped only if every value it can take maps to the colour
 *    map's first entry through a leading run of equal entries.
 *  BC_STEP_FIXED (default): the views' step.
 *  BC_STEP_PER_VOXEL: per ray, step 1 / max_a |d_a| for the unit direction d:
 *    consecutive samples one voxel apart along the ray's dominant axis, at
 *    least one sample in every voxel slice the ray crosses (the discrete ray
 *    casting of Section 2.3.2); samples stay anchored at the cube entry.  The
 *    views' step must still be valid (> 0) and is not used.
 * Errors: BC_E_ARG for an unknown op or step_policy; BC_E_UNSUPPORTED for
 * BC_STEP_PER_VOXEL with BC_OP_COMPOSITE (the composited table is corrected
 * for one step per frame).  bc_render_frame returns BC_E_UNSUPPORTED for
 * learned frames with BC_OP_MIP. */
enum bc_operator { BC_OP_COMPOSITE = 0, BC_OP_MIP = 1 };
enum bc_step_policy { BC_STEP_FIXED = 0, BC_STEP_PER_VOXEL = 1 };
int bc_set_operator(bc_ctx* ctx, int op, int step_policy);

/* Statistics of the last frame; waits for it to finish. */
typedef struct {
  uint64_t nominal_samples;    /* samples taken, up to termination, skipped-empty ones included */
  uint64_t evaluated_samples;  /* samples actually interpolated (and looked up, when compositing) */
  uint32_t n_tiles;            /* (brick, view, 8x8 tile) work items of all passes of the frame */
  int32_t fell_back;           /* learned frame: 1 if it was re-rendered plain, else 0; -1 for a plain frame */
  float psnr_db;               /* learned frame: PSNR (peak 1) of the validation tiles; NaN for a plain frame */
  uint32_t reserved;
} bc_frame_stats;
int bc_get_frame_stats(bc_ctx* ctx, bc_frame_stats* stats);

/* Options (any time after bc_create; they apply from the next frame).
 *  BC_OPT_EMPTY_SKIP (default 1): samples whose interpolation cell cannot reach
 *    a transfer-function entry of non-zero opacity add exactly nothing to their
 *    ray; with 1 they are counted but not evaluated (the image is bit-identical
 *    to 0).  The per-cell classification is recomputed on the device whenever
 *    the opacity-corrected table changes.
 *  BC_OPT_RENDER_WORKGROUPS: workgroups (256 threads) of the persistent
 *    ray-casting launch; default 4 per compute unit.
 *  BC_OPT_SAMPLE_CHUNK (32 or 64, default 32): samples per ray whose
 *    occupancy is gathered before the occupied ones are evaluated.  Images do
 *    not depend on it.
 *  BC_OPT_GRAPH (default 0): 1 captures each frame's kernels once
 *    into a HIP graph (one per per-frame input buffer; captured again when the
 *    view count, frame size, table size, launch options, mode or `out` change)
 *    and replays it; images are identical.  With a graph, timing reports the
 *    whole frame in stage 1 (ray casting) and zero for the other stages.
 *  BC_OPT_XCD_QUEUES (default 1): 1 splits the work items into 8 queues of
 *    whole bricks (brick b in queue b % 8), each served first by the
 *    workgroups of one XCD, so that the eight L2 caches hold different bricks;
 *    0 uses a single queue.  Images do not depend on it.
 *  BC_OPT_TILE_WIDTH (4, 8 or 16; default 8): width in pixels of the screen
 *    tile one wave casts (its 64 rays): 4 x 16, 8 x 8 or 16 x 4 pixels.
 *    Rendering rectangles and work items are counted in these tiles.  Images
 *    do not depend on it.  BC_E_NOMEM (shape unchanged) if the current views
 *    would need more sub-image tiles than planned with this shape.
 * Errors: BC_E_ARG for an unknown option or a value out of range. */
enum bc_option { BC_OPT_EMPTY_SKIP = 0, BC_OPT_RENDER_WORKGROUPS = 1, BC_OPT_SAMPLE_CHUNK = 2, BC_OPT_GRAPH = 3,
                 BC_OPT_XCD_QUEUES = 4, BC_OPT_TILE_WIDTH = 5 };
int bc_set_option(bc_ctx* ctx, int option, int64_t value);

/* Autotuner: renders the current views (plain frames) with every candidate
 * launch shape -- screen tiles of 8 x 8, 16 x 4 and 4 x 16 pixels (those whose
 * work items fit the planned sub-image tiles) times samples per occupancy chunk
 * in {32, 64} times persistent workgroups in {2, 4, 6, 8} per compute unit --
 * for `frames` timed frames each (after one warm-up frame per candidate),
 * measures the ray-casting kernel with HIP events and keeps the fastest;
 * chosen[0] = chunk, chosen[1] = workgroups, chosen[2] = tile width in pixels
 * (chosen may be NULL; else it has 3 entries).  Writes frames into `out` (same
 * contract as bc_render_frame) and waits for them.  The result applies to
 * later frames (also settable with bc_set_option).  Errors: as
 * bc_render_frame; BC_E_ARG for frames outside [1, 64]; BC_E_STATE with
 * learned frames on. */
int bc_autotune(bc_ctx* ctx, float* out, void* stream, int frames, int64_t chosen[3]);

/* Per-stage GPU time, measured with HIP events recorded on the frame's own
 * stream.  bc_enable_timing(ctx, 1) waits for the last frame and opens a new
 * measurement window; each following bc_render_frame (at most 4096 of them)
 * records an event before the set-up kernel, before the ray-casting kernel,
 * before the compositing kernel and after it.  bc_enable_timing(ctx, 2) does
 * the same with only the two events around the ray-casting kernel (each
 * event recorded between dependent kernels costs the frame a few
 * microseconds); set-up and compositing then read zero.
 * bc_enable_timing(ctx, 0) stops recording.  bc_get_timing waits for the last
 * frame and writes the summed milliseconds of the window's frames per stage:
 * ms_out[0] set-up, ms_out[1] ray casting, ms_out[2] compositing; *n_frames
 * (may be NULL) receives the number of frames summed.  Errors: BC_E_STATE on
 * a host-only context, BC_E_ARG for a null ms_out or an enable outside
 * {0, 1, 2}. */
int bc_enable_timing(bc_ctx* ctx, int enable);
int bc_get_timing(bc_ctx* ctx, double ms_out[3], int* n_frames);
/* Whole-frame milliseconds (first event to last) of each frame of the current
 * timing window, in order, at most cap of them (the ray-casting kernel's
 * under bc_enable_timing(ctx, 2)); *n_frames (may be NULL) receives the
 * window's frame count.  Waits for the last frame. */
int bc_get_frame_times(bc_ctx* ctx, double* ms, int cap, int* n_frames);

/* Brick table after bc_load_bricks: per brick the core box lo/hi (6 int32,
 * global voxel coordinates) and the FP8 (scale, offset) (1, 0 otherwise),
 * and the (min, max) of its stored values.  Any of the output arrays may be
 * NULL.  *n receives the brick count; at most cap entries are written. */
int bc_get_bricks(bc_ctx* ctx, int32_t* lo_hi, float* scale_offset, float* min_max, int cap, int* n);

/* Visibility order (front to back brick indices) and rendering rectangles
 * (x0, y0, x1, y1 half-open pixel bounds, already widened to whole screen
 * tiles of the last frame's shape) of `view` in the last frame; waits for it
 * to finish. */
int bc_get_visibility_order(bc_ctx* ctx, int view, int32_t* order, int cap);
int bc_get_rects(bc_ctx* ctx, int view, int32_t* rects, int cap);

/* Copy the stored elements of brick `b` to host memory `dst` of `cap` bytes
 * and report the padded dims.  Layout: the ghosted brick padded to a multiple
 * of 4 per axis, as 4x4x4 micro-blocks in row-major order; a micro-block is 16
 * rows (y, then z) of 5 elements, the row's 4 voxels (x fastest) followed by
 * the first voxel of the next micro-block along x (the last voxel of the
 * padded brick where there is none).  80 elements per micro-block, so
 * mbx*mby*mbz*80 elements in all.  For tests of the layout and the encoders. */
int bc_read_brick(bc_ctx* ctx, int b, void* dst, size_t cap, int32_t padded_dims[3]);

/* ---------------------------------------------------------------------------
 * Learned upsampler (no passage in the paper: an addition that reconstructs a
 * full-resolution, fine-step frame from a half-resolution, coarse-step one).
 * Network: three 3x3 convolutions with zero padding, 4 -> 32 (ReLU) -> 32
 * (ReLU) -> 16, then a 2x2 pixel shuffle (channel 4c + 2dy + dx goes to fine
 * pixel (2i+dy, 2j+dx), channel c) plus the bilinear 2x upsampling of the input
 * (half-pixel centres, clamped).  BF16 operands, FP32 accumulation, FP32
 * master weights.  Parameters: CNN_N_PARAMS = 15056 floats, in the order
 * W1[32][4][3][3] b1[32] W2[32][32][3][3] b2[32] W3[16][32][3][3] b3[16].
 * Images are NHWC float32 RGBA device buffers, 16-byte aligned: coarse
 * n x h x w x 4, fine n x 2h x 2w x 4.
 *
 * bc_cnn_plan: workspace bytes for up to max_n images of max_h x max_w coarse
 *   pixels (parameters, Adam moments, packed BF16 weights, activations,
 *   per-tile partial sums).  BC_E_ARG outside 1 <= max_n <= 64, sizes in
 *   [1, 8192]; BC_E_STATE once bound.
 * bc_cnn_bind: caller-allocated device workspace (256-byte aligned), kept alive
 *   by the caller; BC_E_NOMEM if smaller than planned.
 * bc_cnn_set_weights: copy n = 15056 host floats (and optionally both Adam
 *   moments, else zeros) and the Adam step count; all finite.  For a
 *   checkpoint, bc_cnn_get_weights returns the same four items.
 * bc_cnn_forward: enqueue inference of n coarse images on `stream`.
 * bc_cnn_gradients: gradient of the mean squared error over all fine pixels
 *   and channels with respect to the parameters, into host `grad` (may be NULL),
 *   and the loss into host `loss` (may be NULL); synchronous; no update.
 * bc_cnn_train_step: gradient as above, then one bias-corrected Adam step
 *   (beta 0.9 / 0.999, eps 1e-8, learning rate lr > 0) on `stream`; if `loss` is
 *   non-NULL the call waits and returns the loss before the update.
 * Errors: BC_E_STATE before bind / weights, BC_E_ARG for null or misaligned
 * images, sizes beyond the plan, n != 15056, non-finite values. */
int bc_cnn_plan(bc_ctx* ctx, int max_n, int max_h, int max_w, size_t* bytes);
int bc_cnn_bind(bc_ctx* ctx, void* workspace, size_t bytes);
int bc_cnn_set_weights(bc_ctx* ctx, const float* w, const float* adam_m, const float* adam_v, size_t n, int64_t step);
int bc_cnn_get_weights(bc_ctx* ctx, float* w, float* adam_m, float* adam_v, size_t n, int64_t* step);
int bc_cnn_forward(bc_ctx* ctx, const float* coarse, float* fine, int n, int h, int w, void* stream);
int bc_cnn_gradients(bc_ctx* ctx, const float* coarse, const float* target, int n, int h, int w, float* grad,
                     float* loss);
int bc_cnn_train_step(bc_ctx* ctx, const float* coarse, const float* target, int n, int h, int w, float lr,
                      float* loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BRICKCAST_H */
