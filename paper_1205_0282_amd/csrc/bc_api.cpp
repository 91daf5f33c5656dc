// Host runtime of the bricked ray caster: argument checking, memory planning,
// brick loading, per-frame parameters (read by the set-up kernel from pinned
// host memory) and kernel sequencing.
// The declarations and the contract of every entry point are in
// include/brickcast.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/brickcast.h"
#include "bc_cnn.h"
#include "bc_kernels.h"
#include "bc_types.h"

// Sub-image tiles of bc_render_frame_static: a fixed device array in place of
// the bound sub-image region, for callers that cannot allocate.  Each device
// the library runs on holds its own copy until the process ends.  In host code
// the name is only a stand-in: kernels are given the device address that
// hipGetSymbolAddress returns for it (kept per device below), never the name.
static __device__ __align__(256) float4 scratch[(size_t)BC_STATIC_MAX_TILES * 64];

namespace {

thread_local std::string g_create_error;

// device address of `scratch` on each device, looked up once per device
std::mutex g_scratch_mu;
std::map<int, float4*> g_scratch_ptr;

// looks up the address of `scratch` on `device` (which must be current) the
// first time, then returns the kept one; nullptr on failure
float4* static_scratch(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    if (err) *err = e;
    return nullptr;
  }
  g_scratch_ptr[device] = static_cast<float4*>(ptr);
  return static_cast<float4*>(ptr);
}

struct GraphKey {
  bool learned = false, ess = false, xcd = false;
  int n_views = 0, W = 0, H = 0, K = 0, chunk = 0, wgs = 0, op = 0, step_policy = 0, tile_shift = 0;
  int64_t split = 0;   // learned frames: sub-image tiles set aside for the concurrent validation pass (0: serial)
  const void* out = nullptr;
  const void* sub = nullptr;   // sub-image tiles the launches write
  bool operator==(const GraphKey& o) const {
    return learned == o.learned && ess == o.ess && xcd == o.xcd && n_views == o.n_views && W == o.W && H == o.H && K == o.K &&
           chunk == o.chunk && wgs == o.wgs && op == o.op && step_policy == o.step_policy && split == o.split &&
           tile_shift == o.tile_shift &&
           out == o.out && sub == o.sub;
  }
};
struct GraphSlot {
  hipGraphExec_t exec = nullptr;
  GraphKey key;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxTimedFrames = 4096;
constexpr int kPasses = 3;   // learned frame: coarse, validation, conditional plain

}  // namespace

struct bc_ctx {
  int device = -1;
  std::string err;
  int n_cu = 256;
  // plan
  bool planned = false, bound = false, loaded = false, has_tf = false, has_view = false;
  bc_volume_desc desc{};
  int max_views = 0, max_w = 0, max_h = 0;
  int64_t max_tiles = 0;
  int nb[3] = {0, 0, 0};
  int n_bricks = 0;
  std::vector<BcBrick> bricks;
  size_t elem_bytes = 4, src_elem_bytes = 4;
  size_t bytes[4] = {0, 0, 0, 0};
  size_t off_bricks = 0, off_fin = 0, off_views = 0, off_order = 0, off_rects = 0, off_item_base = 0,
         off_ctr = 0, off_occ = 0, off_item_perm = 0, off_item_entry = 0;
  // a second set of per-pass arrays, for a pass that runs concurrently with
  // another (the validation pass of a learned frame)
  size_t off_views_b = 0, off_order_b = 0, off_rects_b = 0, off_item_base_b = 0, off_item_perm_b = 0,
         off_item_entry_b = 0, off_ctr_b = 0;
  int max_occ_words = 0;
  void* dev[4] = {nullptr, nullptr, nullptr, nullptr};
  // per-frame input ring (pinned host memory, kPasses pass inputs per slot) and events
  BcFrameIn* pinned[2] = {nullptr, nullptr};
  const BcFrameIn* pinned_dev[2] = {nullptr, nullptr};   // the same buffers' device-side addresses
  hipEvent_t slot_done[2] = {nullptr, nullptr};
  bool slot_pending[2] = {false, false};
  int ring = 0;
  hipEvent_t frame_done = nullptr;
  bool frame_pending = false;
  int frame_views = 0;
  // host-source load staging (pinned)
  void* load_staging = nullptr;
  size_t load_staging_bytes = 0;
  // transfer function and views (host copies)
  std::vector<float> tf;
  int K = 0;
  double vmin = 0, vmax = 1, dt_ref = 1;
  std::vector<bc_view> views;
  int64_t view_tiles = 0;          // host bound on the sub-image tiles the views need
  float4* static_sub = nullptr;    // this device's copy of `scratch`
  std::vector<float> occ_key;      // per-frame classification key (sized with the table)
  // kernel launch shape and options
  int render_workgroups = 0;
  // screen tiles of (1 << tile_shift) x (64 >> tile_shift) pixels (8 x 8 by
  // default); the shape of the last frame, for its rectangles
  int tile_shift = 3, frame_tile_shift = 3;
  bool ess = true;
  bool xcd_queues = true;
  int chunk = 32;
  // ray operator and step policy (bc_set_operator)
  int op = BC_OP_COMPOSITE;
  int step_policy = BC_STEP_FIXED;
  // captured frames (one per input slot)
  bool use_graph = false;
  hipStream_t capture_stream = nullptr;
  // learned frames: second stream for the validation pass, and the events
  // that fork it from and join it back to the frame's stream
  hipStream_t aux_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  GraphSlot graphs[2];
  // cell-occupancy bits are valid for this table (opacity-corrected entries)
  bool occ_valid = false;
  std::vector<float> occ_table;
  // learned upsampler: caller-bound workspace (see cnn_layout)
  bool cnn_planned = false, cnn_bound = false, cnn_has_w = false;
  int cnn_max_n = 0, cnn_max_h = 0, cnn_max_w = 0;
  size_t cnn_bytes = 0;
  char* cnn_ws = nullptr;
  int64_t cnn_step = 0;
  std::vector<float> cnn_loss_host;
  // learned frames: coarse render + upsampler, validated on a sparse set of
  // tiles rendered plain; falls back to the plain render below the threshold
  bool learned = false, last_learned = false;
  double coarse_step = 2.0, psnr_threshold = 40.0;
  int val_stride = 8;
  uint64_t frame_counter = 0;
  // per-stage timing: 4 events per frame (before setup, before render, before
  // composite, after composite) recorded on the frame's stream
  bool timing = false;
  bool timing_stages = true;   // all four events per frame, or the two around the ray caster
  std::vector<hipEvent_t> tev;
  int timed_frames = 0;
};

namespace {

int fail(bc_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHECK(c, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail((c), BC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool is_fin(double x) { return std::isfinite(x); }

// row-major 4x4 from OpenGL column-major
void rowmajor(const double* cm, double* rm) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) rm[r * 4 + c] = cm[c * 4 + r];
}

double det4(const double* m) {
  // Laplace expansion over 2x2 minors
  const double s0 = m[0] * m[5] - m[4] * m[1], s1 = m[0] * m[6] - m[4] * m[2];
  const double s2 = m[0] * m[7] - m[4] * m[3], s3 = m[1] * m[6] - m[5] * m[2];
  const double s4 = m[1] * m[7] - m[5] * m[3], s5 = m[2] * m[7] - m[6] * m[3];
  const double c5 = m[10] * m[15] - m[14] * m[11], c4 = m[9] * m[15] - m[13] * m[11];
  const double c3 = m[9] * m[14] - m[13] * m[10], c2 = m[8] * m[15] - m[12] * m[11];
  const double c1 = m[8] * m[14] - m[12] * m[10], c0 = m[8] * m[13] - m[12] * m[9];
  return s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
}

// samples along the cube's diagonal at this step stay at most 2^22, so that
// sample indices are exact in FP32 with a fraction to spare (the ray caster
// rounds half-sample times in FP32)
bool step_fits(const bc_ctx* c, double step) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) d2 += (double)c->desc.global_dims[a] * (double)c->desc.global_dims[a];
  return std::sqrt(d2) / step <= 4194304.0;
}

int check_view(bc_ctx* c, const bc_view& v, int idx) {
  if (v.width < 1 || v.height < 1 || v.width > 16384 || v.height > 16384)
    return fail(c, BC_E_ARG, "view %d: width/height %d x %d outside [1, 16384]", idx, v.width, v.height);
  if (!(is_fin(v.step) && v.step > 0.0)) return fail(c, BC_E_ARG, "view %d: step must be finite and > 0", idx);
  if (c->planned && !step_fits(c, v.step))
    return fail(c, BC_E_ARG, "view %d: step %g takes more than 2^22 samples along the cube's diagonal", idx, v.step);
  if (!(v.ert_threshold > 0.0 && v.ert_threshold <= 1.0))
    return fail(c, BC_E_ARG, "view %d: ert_threshold must be in (0, 1]", idx);
  double M[16], P[16];
  rowmajor(v.modelview, M);
  rowmajor(v.projection, P);
  for (int k = 0; k < 16; ++k)
    if (!is_fin(M[k]) || !is_fin(P[k])) return fail(c, BC_E_ARG, "view %d: non-finite matrix entry", idx);
  if (!(M[12] == 0.0 && M[13] == 0.0 && M[14] == 0.0 && M[15] == 1.0))
    return fail(c, BC_E_ARG, "view %d: modelview bottom row must be (0, 0, 0, 1)", idx);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += M[i * 4 + k] * M[j * 4 + k];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-9)
        return fail(c, BC_E_ARG, "view %d: modelview rotation is not orthonormal", idx);
    }
  const bool persp = P[12] == 0.0 && P[13] == 0.0 && P[14] == -1.0 && P[15] == 0.0;
  const bool ortho = P[12] == 0.0 && P[13] == 0.0 && P[14] == 0.0 && P[15] == 1.0;
  if (!persp && !ortho)
    return fail(c, BC_E_ARG, "view %d: projection is neither perspective nor orthographic", idx);
  if (!(std::fabs(det4(P)) > 0.0)) return fail(c, BC_E_ARG, "view %d: projection is singular", idx);
  return BC_OK;
}

// host bound on the work items (brick, selected screen tile) one view needs
// at a frame size, with one tile of every stride x stride block selected:
// the same rectangles as the device set-up, widened by one tile per side
int64_t view_tiles_bound(const bc_ctx* c, const bc_view& v, int W, int H, int stride);

int64_t view_tiles_bound(const bc_ctx* c, const bc_view& v) { return view_tiles_bound(c, v, v.width, v.height, 1); }

int64_t view_tiles_bound(const bc_ctx* c, const bc_view& v, int W, int H, int stride) {
  double M[16], P[16], PM[16];
  rowmajor(v.modelview, M);
  rowmajor(v.projection, P);
  for (int r = 0; r < 4; ++r)
    for (int col = 0; col < 4; ++col) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += P[r * 4 + k] * M[k * 4 + col];
      PM[r * 4 + col] = s;
    }
  const bool persp = P[14] == -1.0;
  double eye[3];
  for (int a = 0; a < 3; ++a) eye[a] = -((M[a] * M[3] + M[4 + a] * M[7]) + M[8 + a] * M[11]);
  const int sx = c->tile_shift, sy = 6 - c->tile_shift;
  const int TX = (W + (1 << sx) - 1) >> sx, TY = (H + (1 << sy) - 1) >> sy;
  // selected tiles among n consecutive ones, wherever the selection starts
  auto sel = [stride](int64_t n) -> int64_t { return (n + stride - 1) / stride; };
  int64_t total = 0;
  for (const BcBrick& b : c->bricks) {
    bool full = false;
    if (persp) {
      bool inside = true;
      for (int a = 0; a < 3; ++a) inside = inside && eye[a] >= b.lo[a] - 1 && eye[a] <= b.hi[a] + 1;
      full = inside;
    }
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int k = 0; k < 8 && !full; ++k) {
      const double X = (k & 1) ? b.hi[0] : b.lo[0], Y = (k & 2) ? b.hi[1] : b.lo[1], Z = (k & 4) ? b.hi[2] : b.lo[2];
      double cl[4];
      for (int i = 0; i < 4; ++i) cl[i] = PM[i * 4] * X + PM[i * 4 + 1] * Y + PM[i * 4 + 2] * Z + PM[i * 4 + 3];
      if (!(cl[3] > 1e-12)) { full = true; break; }
      const double px = (cl[0] / cl[3] + 1.0) * 0.5 * W - 0.5, py = (1.0 - cl[1] / cl[3]) * 0.5 * H - 0.5;
      xmin = std::min(xmin, px); xmax = std::max(xmax, px);
      ymin = std::min(ymin, py); ymax = std::max(ymax, py);
    }
    if (full) { total += sel(TX) * sel(TY); continue; }
    if (xmax < -2.0 || ymax < -2.0 || xmin > W + 1.0 || ymin > H + 1.0) continue;
    const int x0 = (int)std::max(std::floor(xmin) - 1.0, 0.0), y0 = (int)std::max(std::floor(ymin) - 1.0, 0.0);
    const int x1 = (int)std::min(std::ceil(xmax) + 1.0, (double)(W - 1)), y1 = (int)std::min(std::ceil(ymax) + 1.0, (double)(H - 1));
    if (x1 < x0 || y1 < y0) continue;
    const int tx0 = std::max((x0 >> sx) - 1, 0), ty0 = std::max((y0 >> sy) - 1, 0);
    const int tx1 = std::min((x1 >> sx) + 2, TX), ty1 = std::min((y1 >> sy) + 2, TY);
    total += sel(tx1 - tx0) * sel(ty1 - ty0);
  }
  return total;
}

BcFramePtrs frame_ptrs(bc_ctx* c) {
  char* meta = static_cast<char*>(c->dev[1]);
  BcFramePtrs f{};   // every field set below, or zero
  f.fin = reinterpret_cast<const BcFrameIn*>(meta + c->off_fin);
  f.views = reinterpret_cast<BcViewParams*>(meta + c->off_views);
  f.bricks = reinterpret_cast<const BcBrick*>(meta + c->off_bricks);
  f.order = reinterpret_cast<int32_t*>(meta + c->off_order);
  f.rects = reinterpret_cast<int32_t*>(meta + c->off_rects);
  f.item_base = reinterpret_cast<int32_t*>(meta + c->off_item_base);
  f.item_perm = reinterpret_cast<int32_t*>(meta + c->off_item_perm);
  f.item_entry = reinterpret_cast<int4*>(meta + c->off_item_entry);
  f.n_queues = c->xcd_queues ? 8 : 1;
  f.ctr = reinterpret_cast<BcCounters*>(meta + c->off_ctr);
  f.sub = static_cast<float4*>(c->dev[2]);
  f.pool = c->dev[0];
  f.occ = reinterpret_cast<uint32_t*>(meta + c->off_occ);
  f.ess = c->ess ? 1 : 0;
  f.chunk = c->chunk;
  f.tile_shift = c->tile_shift;
  // the ray caster's waves issue at the raised priority levels (measured
  // 0.8% faster on the bench orbit than the base levels); only a pass that
  // runs beside a more urgent one (a learned frame's coarse pass) is lowered
  f.urgent = 1;
  f.K = c->K;
  f.op = c->op;
  f.step_policy = c->step_policy;
  f.n_bricks = c->n_bricks;
  f.n_views = c->frame_views;
  for (int a = 0; a < 3; ++a) f.gdims[a] = (int32_t)c->desc.global_dims[a];
  f.max_items = c->max_tiles;
  f.storage = c->desc.storage;
  f.width = c->views.empty() ? 0 : c->views[0].width;
  f.height = c->views.empty() ? 0 : c->views[0].height;
  return f;
}

int wait_frame(bc_ctx* c) {
  if (c->frame_pending) {
    HIPCHECK(c, hipEventSynchronize(c->frame_done));
  }
  return BC_OK;
}

struct PassSpec {
  int width, height;
  double step;
  int stride, ox, oy;
  bool reset, conditional;
};

// per-pass input: the views at the pass's size and step, the table (opacity-
// corrected and premultiplied for that step when compositing, the straight
// colour map for maximum intensity projection), and the tile selection
void fill_pass(bc_ctx* c, BcFrameIn* fin, const PassSpec& p) {
  const int n = (int)c->views.size();
  for (int i = 0; i < n; ++i) {
    BcViewIn& vi = fin->views[i];
    std::memcpy(vi.mv, c->views[i].modelview, sizeof vi.mv);
    std::memcpy(vi.pr, c->views[i].projection, sizeof vi.pr);
    vi.width = p.width;
    vi.height = p.height;
    vi.step = p.step;
    vi.tau = c->views[i].ert_threshold;
  }
  fin->n_views = n;
  fin->K = c->K;
  const double scale = (c->K - 1) / (c->vmax - c->vmin);
  fin->tf_scale = (float)scale;
  fin->tf_bias = (float)(-c->vmin * scale);
  fin->tile_stride = p.stride;
  fin->tile_ox = p.ox;
  fin->tile_oy = p.oy;
  fin->reset_counters = p.reset ? 1 : 0;
  fin->conditional = p.conditional ? 1 : 0;
  fin->psnr_threshold = (float)c->psnr_threshold;
  fin->op = c->op;
  fin->step_policy = c->step_policy;
  if (c->op == BC_OP_MIP) {
    for (int k = 0; k < c->K; ++k)
      for (int ch = 0; ch < 4; ++ch) fin->table[k][ch] = c->tf[4 * k + ch];
    return;
  }
  for (int k = 0; k < c->K; ++k) {
    const double a = c->tf[4 * k + 3];
    const double ac = 1.0 - std::pow(1.0 - a, p.step / c->dt_ref);
    fin->table[k][0] = (float)(ac * c->tf[4 * k + 0]);
    fin->table[k][1] = (float)(ac * c->tf[4 * k + 1]);
    fin->table[k][2] = (float)(ac * c->tf[4 * k + 2]);
    fin->table[k][3] = (float)ac;
  }
}

BcFramePtrs pass_ptrs(bc_ctx* c, BcFramePtrs f, int pass, int width, int height) {
  f.fin = reinterpret_cast<const BcFrameIn*>(static_cast<char*>(c->dev[1]) + c->off_fin + sizeof(BcFrameIn) * pass);
  if (f.fin_src) f.fin_src += pass;
  f.width = width;
  f.height = height;
  return f;
}

// the same pass on the second set of per-pass arrays, with the sub-image
// tiles [first, first + cap) of the shared buffer `sub`
BcFramePtrs second_slot(bc_ctx* c, BcFramePtrs f, float4* sub, int64_t first, int64_t cap) {
  char* meta = static_cast<char*>(c->dev[1]);
  f.views = reinterpret_cast<BcViewParams*>(meta + c->off_views_b);
  f.order = reinterpret_cast<int32_t*>(meta + c->off_order_b);
  f.rects = reinterpret_cast<int32_t*>(meta + c->off_rects_b);
  f.item_base = reinterpret_cast<int32_t*>(meta + c->off_item_base_b);
  f.item_perm = reinterpret_cast<int32_t*>(meta + c->off_item_perm_b);
  f.item_entry = reinterpret_cast<int4*>(meta + c->off_item_entry_b);
  f.ctr = reinterpret_cast<BcCounters*>(meta + c->off_ctr_b);
  f.sub = sub + first * 64;
  f.max_items = cap;
  return f;
}

struct CnnLayout {
  size_t w, m, v, g;                 // FP32 parameter vectors
  size_t f1, f2, f3, b3, b2;         // packed fragments: forward 1..3, backward-data 3 and 2
  size_t a1, a2, gy, gz2, gz1;       // BF16 NHWC activations / gradients
  size_t part, loss;                 // per-tile partial sums
  size_t coarse, val;                // learned frames: coarse render, validation tiles
  size_t total;
  int64_t tiles;
};

// fragment bytes: ks * nt * 64 lanes * 8 BF16
constexpr size_t frag_bytes(int ks, int nt) { return (size_t)ks * nt * 64 * 8 * 2; }
constexpr int kPartWidth = 32 * 288 + 32;   // widest per-tile partial (layer 2)

CnnLayout cnn_layout(int n, int h, int w) {
  CnnLayout L;
  size_t m = 0;
  auto take = [&](size_t bytes) { size_t o = m; m = align256(m + bytes); return o; };
  L.w = take(4 * CNN_N_PARAMS);
  L.m = take(4 * CNN_N_PARAMS);
  L.v = take(4 * CNN_N_PARAMS);
  L.g = take(4 * CNN_N_PARAMS);
  L.f1 = take(frag_bytes(2, 2));
  L.f2 = take(frag_bytes(9, 2));
  L.f3 = take(frag_bytes(9, 1));
  L.b3 = take(frag_bytes(5, 2));
  L.b2 = take(frag_bytes(9, 2));
  const size_t px = (size_t)n * h * w;
  L.a1 = take(px * 32 * 2);
  L.a2 = take(px * 32 * 2);
  L.gy = take(px * 16 * 2);
  L.gz2 = take(px * 32 * 2);
  L.gz1 = take(px * 32 * 2);
  L.tiles = (int64_t)n * ((h + 15) / 16) * ((w + 15) / 16);
  L.part = take((size_t)L.tiles * kPartWidth * 4);
  L.loss = take((size_t)L.tiles * 4);
  L.coarse = take(px * 16);
  L.val = take(px * 4 * 16);
  L.total = m;
  return L;
}

int cnn_infer(bc_ctx* c, const CnnLayout& L, const float* coarse, float* fine, int n, int h, int w, hipStream_t st);

}  // namespace

extern "C" {

int bc_create(int hip_device, bc_ctx** out) {
  if (!out) { g_create_error = "bc_create: out is NULL"; return BC_E_ARG; }
  *out = nullptr;
  if (hip_device < -1) { g_create_error = "bc_create: device must be >= -1"; return BC_E_ARG; }
  bc_ctx* c = new bc_ctx();
  c->device = hip_device;
  if (hip_device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || hip_device >= n) {
      g_create_error = std::string("bc_create: no HIP device ") + std::to_string(hip_device) + ": " +
                       (e != hipSuccess ? hipGetErrorString(e) : "index out of range");
      delete c;
      return BC_E_HIP;
    }
    hipDeviceProp_t prop;
    if (hipSetDevice(hip_device) != hipSuccess || hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
      g_create_error = "bc_create: cannot query device";
      delete c;
      return BC_E_HIP;
    }
    c->n_cu = prop.multiProcessorCount;
    c->render_workgroups = c->n_cu * 4;
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) {
      // host-coherent: the set-up kernel reads the pass inputs from here, and
      // no GPU cache may serve it an earlier frame's copy of a slot
      ok = hipHostMalloc(reinterpret_cast<void**>(&c->pinned[i]), sizeof(BcFrameIn) * kPasses, hipHostMallocCoherent) ==
           hipSuccess;
      void* dp = nullptr;
      ok = ok && hipHostGetDevicePointer(&dp, c->pinned[i], 0) == hipSuccess;
      c->pinned_dev[i] = static_cast<const BcFrameIn*>(dp);
      ok = ok && hipEventCreateWithFlags(&c->slot_done[i], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipEventCreateWithFlags(&c->frame_done, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      g_create_error = "bc_create: cannot allocate pinned frame buffers / events";
      bc_destroy(c);
      return BC_E_HIP;
    }
    hipError_t se = hipSuccess;
    c->static_sub = static_scratch(hip_device, &se);
    if (!c->static_sub) {
      g_create_error = std::string("bc_create: hipGetSymbolAddress(scratch): ") + hipGetErrorString(se);
      bc_destroy(c);
      return BC_E_HIP;
    }
  }
  *out = c;
  return BC_OK;
}

void bc_destroy(bc_ctx* c) {
  if (!c) return;
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    if (c->frame_pending) (void)hipEventSynchronize(c->frame_done);
    for (int i = 0; i < 2; ++i) {
      if (c->slot_done[i]) (void)hipEventDestroy(c->slot_done[i]);
      if (c->pinned[i]) (void)hipHostFree(c->pinned[i]);
    }
    if (c->frame_done) (void)hipEventDestroy(c->frame_done);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    for (GraphSlot& g : c->graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    if (c->load_staging) (void)hipHostFree(c->load_staging);
  }
  delete c;
}

const char* bc_last_error(const bc_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int bc_plan(bc_ctx* c, const bc_volume_desc* d, int max_views, int max_w, int max_h, int64_t max_tiles,
            size_t bytes_out[4]) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!d || !bytes_out) return fail(c, BC_E_ARG, "bc_plan: null desc or bytes_out");
  for (int a = 0; a < 3; ++a) {
    if (d->global_dims[a] < 1 || d->global_dims[a] > (1 << 20))
      return fail(c, BC_E_ARG, "bc_plan: global_dims[%d] = %lld outside [1, 2^20]", a, (long long)d->global_dims[a]);
    if (d->share_lo[a] < 0 || d->share_hi[a] > d->global_dims[a] || d->share_lo[a] >= d->share_hi[a])
      return fail(c, BC_E_ARG, "bc_plan: share [%lld, %lld) on axis %d is empty or outside the cube",
                  (long long)d->share_lo[a], (long long)d->share_hi[a], a);
    if (d->brick_dims[a] < 1 || d->brick_dims[a] > 1024)
      return fail(c, BC_E_ARG, "bc_plan: brick_dims[%d] = %d outside [1, 1024]", a, d->brick_dims[a]);
  }
  if (d->ghost != 1) return fail(c, BC_E_ARG, "bc_plan: ghost must be 1");
  if (d->storage < 0 || d->storage > 2) return fail(c, BC_E_ARG, "bc_plan: unknown storage %d", d->storage);
  if (d->src_dtype != BC_F32 && d->src_dtype != BC_F16)
    return fail(c, BC_E_ARG, "bc_plan: src_dtype must be BC_F32 or BC_F16");
  if (max_views < 1 || max_views > BC_MAX_VIEWS) return fail(c, BC_E_ARG, "bc_plan: max_views must be in [1, 4]");
  if (max_w < 1 || max_h < 1 || max_w > 16384 || max_h > 16384)
    return fail(c, BC_E_ARG, "bc_plan: max_w/max_h outside [1, 16384]");
  if (max_tiles < 0) return fail(c, BC_E_ARG, "bc_plan: max_tiles must be >= 0");
  int nb[3];
  int64_t nbt = 1;
  for (int a = 0; a < 3; ++a) {
    const int64_t ext = d->share_hi[a] - d->share_lo[a];
    nb[a] = (int)((ext + d->brick_dims[a] - 1) / d->brick_dims[a]);
    nbt *= nb[a];
  }
  if (nbt > BC_MAX_BRICKS) return fail(c, BC_E_ARG, "bc_plan: %lld bricks exceed the limit of %d", (long long)nbt, BC_MAX_BRICKS);
  {
    // offsets and buffer ranges inside a brick are 32-bit: its stored form
    // (micro-blocks of BC_MB_ELEMS elements over the ghosted box) must stay
    // below 4 GiB
    int64_t mbs = 1;
    for (int a = 0; a < 3; ++a) mbs *= (std::min<int64_t>(d->brick_dims[a], d->share_hi[a] - d->share_lo[a]) + 2 + 3) / 4;
    const int64_t eb = d->storage == BC_F32 ? 4 : (d->storage == BC_F16 ? 2 : 1);
    if (mbs * BC_MB_ELEMS * eb >= (int64_t(1) << 32))
      return fail(c, BC_E_ARG, "bc_plan: a %dx%dx%d brick takes %lld bytes in this storage, 4 GiB or more", d->brick_dims[0],
                  d->brick_dims[1], d->brick_dims[2], (long long)(mbs * BC_MB_ELEMS * eb));
  }
  if (c->bound) return fail(c, BC_E_STATE, "bc_plan: memory already bound to this context");
  c->desc = *d;
  c->max_views = max_views;
  c->max_w = max_w;
  c->max_h = max_h;
  for (int a = 0; a < 3; ++a) c->nb[a] = nb[a];
  c->n_bricks = (int)nbt;
  c->elem_bytes = d->storage == BC_F32 ? 4 : (d->storage == BC_F16 ? 2 : 1);
  c->src_elem_bytes = d->src_dtype == BC_F32 ? 4 : 2;
  c->bricks.assign(c->n_bricks, BcBrick{});
  int64_t off = 0, occ_words = 0, max_words = 0;
  size_t max_region = 0;
  for (int bz = 0; bz < nb[2]; ++bz)
    for (int by = 0; by < nb[1]; ++by)
      for (int bx = 0; bx < nb[0]; ++bx) {
        BcBrick& b = c->bricks[bx + nb[0] * (by + nb[1] * bz)];
        const int bi[3] = {bx, by, bz};
        int64_t region = 1;
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = (int32_t)(d->share_lo[a] + (int64_t)bi[a] * d->brick_dims[a]);
          b.hi[a] = (int32_t)std::min<int64_t>(b.lo[a] + d->brick_dims[a], d->share_hi[a]);
          b.gdim[a] = ((b.hi[a] - b.lo[a] + 2) + 3) / 4 * 4;
          b.mb[a] = b.gdim[a] / 4;
          region *= (b.hi[a] - b.lo[a] + 2);
        }
        b.offset = off;
        b.scale = 1.0f;
        b.offs = 0.0f;
        off += (int64_t)b.mb[0] * b.mb[1] * b.mb[2] * BC_MB_ELEMS;
        // interpolation cells per axis: core + 1 (between ghosted voxels i, i+1)
        b.occ_w[0] = (b.hi[0] - b.lo[0] + 1 + 3) / 4;
        b.occ_w[1] = (b.hi[1] - b.lo[1] + 1 + 3) / 4;
        b.occ_w[2] = (b.hi[2] - b.lo[2] + 1 + 1) / 2;
        b.occ_offset = occ_words;
        const int64_t words = (int64_t)b.occ_w[0] * b.occ_w[1] * b.occ_w[2];
        occ_words += words;
        max_words = std::max<int64_t>(max_words, words);
        max_region = std::max(max_region, (size_t)region);
      }
  // screen tiles of a frame, for the largest count over the tile shapes
  int64_t tiles_frame = 0;
  for (int s = 2; s <= 4; ++s)
    tiles_frame = std::max<int64_t>(tiles_frame, (int64_t)((max_w + (1 << s) - 1) >> s) *
                                                     ((max_h + (1 << (6 - s)) - 1) >> (6 - s)));
  if (max_tiles == 0) {
    // every brick over the whole frame when that is small, else a bound on how
    // many brick rectangles overlap a screen tile
    const int64_t full = (int64_t)max_views * tiles_frame * nbt;
    max_tiles = full <= (int64_t(1) << 18)
                    ? full
                    : (int64_t)max_views * tiles_frame * std::min<int64_t>(nbt, 2 * ((int64_t)nb[0] + nb[1] + nb[2]) + 4);
  }
  c->max_tiles = max_tiles;
  c->bytes[0] = align256((size_t)off * c->elem_bytes);
  size_t m = 0;
  c->off_bricks = m; m = align256(m + sizeof(BcBrick) * c->n_bricks);
  c->off_fin = m; m = align256(m + sizeof(BcFrameIn) * kPasses);
  c->off_views = m; m = align256(m + sizeof(BcViewParams) * BC_MAX_VIEWS);
  c->off_order = m; m = align256(m + sizeof(int32_t) * BC_MAX_VIEWS * c->n_bricks);
  c->off_rects = m; m = align256(m + sizeof(int32_t) * 4 * BC_MAX_VIEWS * c->n_bricks);
  c->off_item_base = m; m = align256(m + sizeof(int32_t) * (BC_MAX_VIEWS * c->n_bricks + 1));
  c->off_item_perm = m; m = align256(m + sizeof(int32_t) * (BC_MAX_VIEWS * c->n_bricks + 1));
  c->off_item_entry = m; m = align256(m + sizeof(int4) * BC_MAX_VIEWS * c->n_bricks);
  c->off_ctr = m; m = align256(m + sizeof(BcCounters));
  c->off_views_b = m; m = align256(m + sizeof(BcViewParams) * BC_MAX_VIEWS);
  c->off_order_b = m; m = align256(m + sizeof(int32_t) * BC_MAX_VIEWS * c->n_bricks);
  c->off_rects_b = m; m = align256(m + sizeof(int32_t) * 4 * BC_MAX_VIEWS * c->n_bricks);
  c->off_item_base_b = m; m = align256(m + sizeof(int32_t) * (BC_MAX_VIEWS * c->n_bricks + 1));
  c->off_item_perm_b = m; m = align256(m + sizeof(int32_t) * (BC_MAX_VIEWS * c->n_bricks + 1));
  c->off_item_entry_b = m; m = align256(m + sizeof(int4) * BC_MAX_VIEWS * c->n_bricks);
  c->off_ctr_b = m; m = align256(m + sizeof(BcCounters));
  c->off_occ = m; m = align256(m + sizeof(uint32_t) * (size_t)occ_words);
  c->bytes[1] = m;
  c->max_occ_words = (int)max_words;
  c->bytes[2] = align256((size_t)max_tiles * 64 * 16);
  c->bytes[3] = align256(max_region * c->src_elem_bytes);
  for (int i = 0; i < 4; ++i) bytes_out[i] = c->bytes[i];
  c->planned = true;
  c->loaded = false;
  c->occ_valid = false;
  if (c->has_view) {
    int64_t tiles = 0;
    for (const bc_view& v : c->views) tiles += view_tiles_bound(c, v);
    c->view_tiles = tiles;
  }
  return BC_OK;
}

int bc_bind_memory(bc_ctx* c, void* const ptrs[4], const size_t sizes[4]) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_bind_memory: host-only context");
  if (!c->planned) return fail(c, BC_E_STATE, "bc_bind_memory: call bc_plan first");
  if (!ptrs || !sizes) return fail(c, BC_E_ARG, "bc_bind_memory: null arrays");
  for (int i = 0; i < 4; ++i) {
    if (!ptrs[i]) return fail(c, BC_E_ARG, "bc_bind_memory: region %d is NULL", i);
    if (reinterpret_cast<uintptr_t>(ptrs[i]) & 255) return fail(c, BC_E_ARG, "bc_bind_memory: region %d not 256-byte aligned", i);
    if (sizes[i] < c->bytes[i])
      return fail(c, BC_E_NOMEM, "bc_bind_memory: region %d has %zu bytes, %zu planned", i, sizes[i], c->bytes[i]);
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptrs[i]) != hipSuccess || attr.type != hipMemoryTypeDevice || attr.device != c->device) {
      (void)hipGetLastError();
      return fail(c, BC_E_ARG, "bc_bind_memory: region %d is not device memory on device %d", i, c->device);
    }
  }
  HIPCHECK(c, hipSetDevice(c->device));
  for (int i = 0; i < 4; ++i) c->dev[i] = ptrs[i];
  char* meta = static_cast<char*>(c->dev[1]);
  HIPCHECK(c, hipMemcpy(meta + c->off_bricks, c->bricks.data(), sizeof(BcBrick) * c->n_bricks, hipMemcpyHostToDevice));
  c->bound = true;
  c->loaded = false;
  return BC_OK;
}

int bc_load_bricks(bc_ctx* c, const void* src, const int64_t strides[3], int src_on_device) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!c->bound) return fail(c, BC_E_STATE, "bc_load_bricks: bind memory first");
  if (!src || !strides) return fail(c, BC_E_ARG, "bc_load_bricks: null src or strides");
  const bc_volume_desc& d = c->desc;
  int64_t box_lo[3], box_hi[3];
  for (int a = 0; a < 3; ++a) {
    box_lo[a] = std::max<int64_t>(d.share_lo[a] - 1, 0);
    box_hi[a] = std::min<int64_t>(d.share_hi[a] + 1, d.global_dims[a]);
  }
  const int64_t ex = box_hi[0] - box_lo[0], ey = box_hi[1] - box_lo[1];
  if (strides[0] < 1 || strides[1] < ex * strides[0] || strides[2] < ey * strides[1])
    return fail(c, BC_E_ARG, "bc_load_bricks: strides (%lld, %lld, %lld) smaller than the source box rows/planes",
                (long long)strides[0], (long long)strides[1], (long long)strides[2]);
  HIPCHECK(c, hipSetDevice(c->device));
  (void)wait_frame(c);
  char* meta = static_cast<char*>(c->dev[1]);
  BcBrick* dbricks = reinterpret_cast<BcBrick*>(meta + c->off_bricks);
  BcCounters* ctr = reinterpret_cast<BcCounters*>(meta + c->off_ctr);
  hipStream_t st = nullptr;
  HIPCHECK(c, bc_launch_init_minmax(ctr, c->n_bricks, st));
  // launch bounds: the largest brick's ghosted rows (y * z) and rows of
  // micro-blocks along x (y * z in micro-blocks)
  int max_rows = 0;
  int64_t max_mb_rows = 0;
  for (const BcBrick& hb : c->bricks) {
    max_rows = std::max(max_rows, (hb.hi[1] - hb.lo[1] + 2) * (hb.hi[2] - hb.lo[2] + 2));
    max_mb_rows = std::max<int64_t>(max_mb_rows, (int64_t)hb.mb[1] * hb.mb[2]);
  }
  if (src_on_device) {
    // the whole share is on the device: every brick in one launch per step
    BcLoadSrc s;
    s.dtype = d.src_dtype == BC_F32 ? 0 : 1;
    s.ptr = src;
    for (int a = 0; a < 3; ++a) {
      s.dims[a] = (int32_t)d.global_dims[a];
      s.strides[a] = strides[a];
      s.origin[a] = (int32_t)box_lo[a];
    }
    HIPCHECK(c, bc_launch_minmax(s, dbricks, 0, c->n_bricks, max_rows, ctr, st));
    HIPCHECK(c, bc_launch_finalize(dbricks, ctr, 0, c->n_bricks, d.storage, st));
    HIPCHECK(c, bc_launch_encode(s, dbricks, 0, c->n_bricks, max_mb_rows, d.storage, c->dev[0], st));
  }
  // a host source goes through the load scratch region one brick at a time
  for (int b = 0; b < c->n_bricks && !src_on_device; ++b) {
    const BcBrick& hb = c->bricks[b];
    BcLoadSrc s;
    s.dtype = d.src_dtype == BC_F32 ? 0 : 1;
    for (int a = 0; a < 3; ++a) s.dims[a] = (int32_t)d.global_dims[a];
    {
      // gather the brick's ghosted region (clamped to the cube) into pinned
      // staging, then copy it into the scratch region
      int64_t rlo[3], rhi[3];
      for (int a = 0; a < 3; ++a) {
        rlo[a] = std::max<int64_t>(hb.lo[a] - 1, 0);
        rhi[a] = std::min<int64_t>(hb.hi[a] + 1, d.global_dims[a]);
      }
      const int64_t rx = rhi[0] - rlo[0], ry = rhi[1] - rlo[1], rz = rhi[2] - rlo[2];
      const size_t need = (size_t)(rx * ry * rz) * c->src_elem_bytes;
      if (need > c->bytes[3]) return fail(c, BC_E_NOMEM, "bc_load_bricks: scratch region too small");
      if (c->load_staging_bytes < need) {
        if (c->load_staging) (void)hipHostFree(c->load_staging);
        c->load_staging = nullptr;
        HIPCHECK(c, hipHostMalloc(&c->load_staging, c->bytes[3], hipHostMallocDefault));
        c->load_staging_bytes = c->bytes[3];
      }
      const char* base = static_cast<const char*>(src);
      char* dst = static_cast<char*>(c->load_staging);
      const size_t eb = c->src_elem_bytes;
      for (int64_t z = 0; z < rz; ++z)
        for (int64_t y = 0; y < ry; ++y) {
          const char* row = base + (((rlo[2] + z - box_lo[2]) * strides[2] + (rlo[1] + y - box_lo[1]) * strides[1] +
                                     (rlo[0] - box_lo[0]) * strides[0]) * eb);
          char* o = dst + ((z * ry + y) * rx) * eb;
          if (strides[0] == 1) {
            std::memcpy(o, row, rx * eb);
          } else {
            for (int64_t x = 0; x < rx; ++x) std::memcpy(o + x * eb, row + x * strides[0] * eb, eb);
          }
        }
      HIPCHECK(c, hipMemcpy(c->dev[3], c->load_staging, need, hipMemcpyHostToDevice));
      s.ptr = c->dev[3];
      s.strides[0] = 1;
      s.strides[1] = rx;
      s.strides[2] = rx * ry;
      for (int a = 0; a < 3; ++a) s.origin[a] = (int32_t)rlo[a];
    }
    HIPCHECK(c, bc_launch_minmax(s, dbricks, b, 1, max_rows, ctr, st));
    HIPCHECK(c, bc_launch_finalize(dbricks, ctr, b, 1, d.storage, st));
    HIPCHECK(c, bc_launch_encode(s, dbricks, b, 1, max_mb_rows, d.storage, c->dev[0], st));
    HIPCHECK(c, hipStreamSynchronize(st));
  }
  HIPCHECK(c, hipStreamSynchronize(st));
  HIPCHECK(c, hipMemcpy(c->bricks.data(), dbricks, sizeof(BcBrick) * c->n_bricks, hipMemcpyDeviceToHost));
  c->loaded = true;
  c->occ_valid = false;
  return BC_OK;
}

int bc_set_transfer_function(bc_ctx* c, const float* rgba, int K, double vmin, double vmax, double dt_ref) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!rgba) return fail(c, BC_E_ARG, "bc_set_transfer_function: rgba is NULL");
  if (K < 2 || K > BC_MAX_K) return fail(c, BC_E_ARG, "bc_set_transfer_function: K = %d outside [2, %d]", K, BC_MAX_K);
  if (!is_fin(vmin) || !is_fin(vmax) || !(vmin < vmax))
    return fail(c, BC_E_ARG, "bc_set_transfer_function: need finite vmin < vmax");
  if (!(is_fin(dt_ref) && dt_ref > 0.0)) return fail(c, BC_E_ARG, "bc_set_transfer_function: dt_ref must be > 0");
  for (int i = 0; i < 4 * K; ++i)
    if (!(rgba[i] >= 0.0f && rgba[i] <= 1.0f))
      return fail(c, BC_E_ARG, "bc_set_transfer_function: entry %d channel %d = %g outside [0, 1]", i / 4, i % 4, (double)rgba[i]);
  c->tf.assign(rgba, rgba + 4 * K);
  c->occ_key.reserve(K + 4);
  c->K = K;
  c->vmin = vmin;
  c->vmax = vmax;
  c->dt_ref = dt_ref;
  c->has_tf = true;
  return BC_OK;
}

int bc_set_view(bc_ctx* c, const bc_view* views, int n) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!views) return fail(c, BC_E_ARG, "bc_set_view: views is NULL");
  if (n < 1 || n > BC_MAX_VIEWS) return fail(c, BC_E_ARG, "bc_set_view: n_views = %d outside [1, 4]", n);
  if (c->planned && n > c->max_views) return fail(c, BC_E_ARG, "bc_set_view: %d views exceed the planned %d", n, c->max_views);
  for (int i = 0; i < n; ++i) {
    int r = check_view(c, views[i], i);
    if (r) return r;
    if (views[i].width != views[0].width || views[i].height != views[0].height || views[i].step != views[0].step ||
        views[i].ert_threshold != views[0].ert_threshold)
      return fail(c, BC_E_ARG, "bc_set_view: all views must share width, height, step and ert_threshold");
    if (c->planned && (views[i].width > c->max_w || views[i].height > c->max_h))
      return fail(c, BC_E_ARG, "bc_set_view: frame %d x %d exceeds the planned %d x %d", views[i].width,
                  views[i].height, c->max_w, c->max_h);
  }
  if (c->planned) {
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) tiles += view_tiles_bound(c, views[i]);
    if (tiles > c->max_tiles)
      return fail(c, BC_E_NOMEM, "bc_set_view: the views need up to %lld sub-image tiles, %lld planned",
                  (long long)tiles, (long long)c->max_tiles);
  }
  {
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) tiles += view_tiles_bound(c, views[i]);
    c->view_tiles = tiles;
  }
  c->views.assign(views, views + n);
  c->has_view = true;
  return BC_OK;
}

}  // extern "C"

namespace {

// One frame: bc_render_frame with the bound sub-image region, or
// bc_render_frame_static (no_alloc) with this device's `scratch`.  `sub` holds
// sub_cap tiles.  With no_alloc nothing is allocated on the host or the device:
// the kernels are launched directly (no graph of the library's own, since
// instantiating one allocates) and the frame is not timed (timing creates its
// events on demand).
int render_impl(bc_ctx* c, float* out, void* stream, float4* sub, int64_t sub_cap, bool no_alloc) {
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_render_frame: host-only context");
  if (!c->bound || !c->loaded) return fail(c, BC_E_STATE, "bc_render_frame: bricks not loaded");
  if (!c->has_tf) return fail(c, BC_E_STATE, "bc_render_frame: no transfer function");
  if (!c->has_view) return fail(c, BC_E_STATE, "bc_render_frame: no view");
  if (!out) return fail(c, BC_E_ARG, "bc_render_frame: out is NULL");
  if (reinterpret_cast<uintptr_t>(out) & 15) return fail(c, BC_E_ARG, "bc_render_frame: out not 16-byte aligned");
  if (c->view_tiles > sub_cap)
    return fail(c, BC_E_NOMEM, "bc_render_frame: the views need up to %lld sub-image tiles, %lld available",
                (long long)c->view_tiles, (long long)sub_cap);
  // (views set before the plan were not checked against the cube)
  if (!step_fits(c, c->views[0].step) || (c->learned && !step_fits(c, c->coarse_step)))
    return fail(c, BC_E_ARG, "bc_render_frame: the step takes more than 2^22 samples along the cube's diagonal");
  const int n = (int)c->views.size();
  const int W = c->views[0].width, H = c->views[0].height;
  if (c->learned) {
    if (!c->cnn_bound || !c->cnn_has_w)
      return fail(c, BC_E_STATE, "bc_render_frame: learned frames need the upsampler workspace and weights");
    if ((W & 1) || (H & 1)) return fail(c, BC_E_ARG, "bc_render_frame: learned frames need an even width and height");
    if (n > c->cnn_max_n || W / 2 > c->cnn_max_w || H / 2 > c->cnn_max_h)
      return fail(c, BC_E_ARG, "bc_render_frame: %d views of %d x %d exceed the upsampler plan", n, W, H);
    if (c->op != BC_OP_COMPOSITE)
      return fail(c, BC_E_UNSUPPORTED, "bc_render_frame: learned frames are trained on composited images only");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHECK(c, hipSetDevice(c->device));
  const int slot = c->ring;
  c->ring ^= 1;
  if (c->slot_pending[slot]) HIPCHECK(c, hipEventSynchronize(c->slot_done[slot]));
  BcFrameIn* pins = c->pinned[slot];
  char* meta = static_cast<char*>(c->dev[1]);
  const int passes = c->learned ? kPasses : 1;
  const double dt = c->views[0].step;
  ++c->frame_counter;
  for (int ps = 0; ps < passes; ++ps) {
    const bool coarse = c->learned && ps == 0;
    PassSpec spec;
    spec.width = coarse ? W / 2 : W;
    spec.height = coarse ? H / 2 : H;
    spec.step = coarse ? c->coarse_step : dt;
    spec.stride = (c->learned && ps == 1) ? c->val_stride : 1;
    // validation tiles move from frame to frame (stratified: one per stride x stride block)
    const uint64_t h = c->frame_counter * 0x9E3779B97F4A7C15ull;
    spec.ox = spec.stride > 1 ? (int)((h >> 32) % (uint64_t)spec.stride) : 0;
    spec.oy = spec.stride > 1 ? (int)((h >> 16) % (uint64_t)spec.stride) : 0;
    spec.reset = ps == 0;
    spec.conditional = c->learned && ps == 2;
    fill_pass(c, pins + ps, spec);
  }
  const size_t fin_bytes = offsetof(BcFrameIn, table) + sizeof(float) * 4 * c->K;
  c->frame_views = n;
  c->frame_tile_shift = c->tile_shift;
  // empty-space classification depends only on which table entries matter
  // (non-zero opacity; for maximum intensity projection, different from the
  // first entry) and on the value-to-table mapping: redo it when that changes
  bool classify = false;
  if (c->ess) {
    // (sized for this table by bc_set_transfer_function: no allocation here)
    std::vector<float>& key = c->occ_key;
    key.resize(c->K + 4);
    key[0] = (float)c->K;
    key[1] = pins[0].tf_scale;
    key[2] = pins[0].tf_bias;
    key[3] = (float)c->op;
    const float* e0 = pins[0].table[0];
    for (int k = 0; k < c->K; ++k) {
      const float* e = pins[0].table[k];
      const bool m = c->op == BC_OP_MIP ? (e[0] != e0[0] || e[1] != e0[1] || e[2] != e0[2] || e[3] != e0[3])
                                         : e[3] != 0.0f;
      key[4 + k] = m ? 1.0f : 0.0f;
    }
    classify = !c->occ_valid || c->occ_table != key;
    if (classify) {
      c->occ_table = key;
      c->occ_valid = true;
    }
  }
  // learned frames: sub-image tiles for a concurrent validation pass, if the
  // coarse pass and the validation pass fit the buffer together (else the
  // passes run one after the other)
  int64_t split = 0;
  if (c->learned) {
    int64_t coarse_tiles = 0, val_tiles = 0;
    for (int i = 0; i < n; ++i) {
      coarse_tiles += view_tiles_bound(c, c->views[i], W / 2, H / 2, 1);
      val_tiles += view_tiles_bound(c, c->views[i], W, H, c->val_stride);
    }
    if (val_tiles > 0 && coarse_tiles + val_tiles <= sub_cap) split = val_tiles;
  }
  hipEvent_t* ev = nullptr;
  if (c->timing && !no_alloc && c->timed_frames < kMaxTimedFrames) {
    const size_t need = 4 * (size_t)(c->timed_frames + 1);
    while (c->tev.size() < need) {
      hipEvent_t e;
      HIPCHECK(c, hipEventCreate(&e));
      c->tev.push_back(e);
    }
    ev = &c->tev[4 * (size_t)c->timed_frames];
    ++c->timed_frames;
  }
  BcFramePtrs f = frame_ptrs(c);
  f.sub = sub;
  f.max_items = sub_cap;
  // each pass's set-up kernel copies that pass's inputs from the slot
  f.fin_src = c->pinned_dev[slot];
  f.fin_bytes = (int32_t)fin_bytes;
  if (classify) {
    HIPCHECK(c, hipMemcpyAsync(meta + c->off_fin, pins, fin_bytes, hipMemcpyHostToDevice, st));
    HIPCHECK(c, bc_launch_classify(f, c->max_occ_words, st));
  }
  // the frame: the kernels of every pass (each pass's set-up kernel first
  // copies the pass inputs from the pinned slot)
  auto enqueue = [&](hipStream_t s, hipEvent_t* e) -> int {
    if (e && c->timing_stages) HIPCHECK(c, hipEventRecord(e[0], s));
    if (!c->learned) {
      HIPCHECK(c, bc_launch_setup(f, s));
      if (e) HIPCHECK(c, hipEventRecord(e[1], s));
      HIPCHECK(c, bc_launch_render(f, c->render_workgroups, s));
      if (e) HIPCHECK(c, hipEventRecord(e[2], s));
      HIPCHECK(c, bc_launch_composite(f, reinterpret_cast<float4*>(out), s));
    } else {
      const CnnLayout L = cnn_layout(c->cnn_max_n, c->cnn_max_h, c->cnn_max_w);
      float* coarse_img = reinterpret_cast<float*>(c->cnn_ws + L.coarse);
      float* val_img = reinterpret_cast<float*>(c->cnn_ws + L.val);
      BcFramePtrs fc = pass_ptrs(c, f, 0, W / 2, H / 2);
      BcFramePtrs fv = pass_ptrs(c, f, 1, W, H);
      if (split > 0) {
        // the validation pass has few work items, each a long walk through a
        // brick: it runs on the second stream, on its own arrays, sub-image
        // tiles and workgroups, while the coarse pass and the network run
        const int val_wgs = (int)std::min<int64_t>((split + 3) / 4, std::max(c->render_workgroups / 4, 1));
        const int main_wgs = std::max(c->render_workgroups - val_wgs, 1);
        BcFramePtrs fvb = second_slot(c, fv, sub, sub_cap - split, split);
        // few long items that gate the frame, ahead of the whole coarse pass
        fvb.urgent = 1;
        fc.urgent = 0;
        fc.max_items = sub_cap - split;
        HIPCHECK(c, hipEventRecord(c->fork_ev, s));
        HIPCHECK(c, hipStreamWaitEvent(c->aux_stream, c->fork_ev, 0));
        HIPCHECK(c, bc_launch_setup(fvb, c->aux_stream));
        HIPCHECK(c, bc_launch_render(fvb, val_wgs, c->aux_stream));
        HIPCHECK(c, bc_launch_composite(fvb, reinterpret_cast<float4*>(val_img), c->aux_stream));
        HIPCHECK(c, hipEventRecord(c->join_ev, c->aux_stream));
        HIPCHECK(c, bc_launch_setup(fc, s));
        HIPCHECK(c, bc_launch_render(fc, main_wgs, s));
        HIPCHECK(c, bc_launch_composite(fc, reinterpret_cast<float4*>(coarse_img), s));
        if (e) HIPCHECK(c, hipEventRecord(e[1], s));
        int r = cnn_infer(c, L, coarse_img, out, n, H / 2, W / 2, s);
        if (r) return r;
        if (e) HIPCHECK(c, hipEventRecord(e[2], s));
        HIPCHECK(c, hipStreamWaitEvent(s, c->join_ev, 0));
      } else {
        HIPCHECK(c, bc_launch_setup(fc, s));
        HIPCHECK(c, bc_launch_render(fc, c->render_workgroups, s));
        HIPCHECK(c, bc_launch_composite(fc, reinterpret_cast<float4*>(coarse_img), s));
        if (e) HIPCHECK(c, hipEventRecord(e[1], s));
        int r = cnn_infer(c, L, coarse_img, out, n, H / 2, W / 2, s);
        if (r) return r;
        if (e) HIPCHECK(c, hipEventRecord(e[2], s));
        HIPCHECK(c, bc_launch_setup(fv, s));
        HIPCHECK(c, bc_launch_render(fv, c->render_workgroups, s));
        HIPCHECK(c, bc_launch_composite(fv, reinterpret_cast<float4*>(val_img), s));
      }
      // the decision is written to the first set of counters, which the
      // conditional pass reads
      HIPCHECK(c, bc_launch_psnr(fv, reinterpret_cast<const float4*>(val_img), reinterpret_cast<const float4*>(out), s));
      BcFramePtrs fp = pass_ptrs(c, f, 2, W, H);
      HIPCHECK(c, bc_launch_setup(fp, s));
      HIPCHECK(c, bc_launch_render(fp, c->render_workgroups, s));
      HIPCHECK(c, bc_launch_composite(fp, reinterpret_cast<float4*>(out), s));
    }
    if (e && c->timing_stages) HIPCHECK(c, hipEventRecord(e[3], s));
    return BC_OK;
  };
  if (!c->use_graph || no_alloc) {
    int r = enqueue(st, ev);
    if (r) return r;
  } else {
    // one captured graph per input slot (its copies read that slot's pinned
    // buffer); re-captured when anything baked into the launches changes
    GraphKey key;
    key.learned = c->learned;
    key.n_views = n;
    key.W = W;
    key.H = H;
    key.K = c->K;
    key.chunk = c->chunk;
    key.ess = c->ess;
    key.wgs = c->render_workgroups;
    key.xcd = c->xcd_queues;
    key.op = c->op;
    key.step_policy = c->step_policy;
    key.tile_shift = c->tile_shift;
    key.split = split;
    key.out = out;
    key.sub = sub;
    GraphSlot& g = c->graphs[slot];
    if (!g.exec || !(g.key == key)) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
      hipGraph_t graph = nullptr;
      HIPCHECK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
      int r = enqueue(c->capture_stream, nullptr);
      hipError_t ec = hipStreamEndCapture(c->capture_stream, &graph);
      if (r) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
      }
      if (ec != hipSuccess) return fail(c, BC_E_HIP, "bc_render_frame: graph capture: %s", hipGetErrorString(ec));
      ec = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ec != hipSuccess) {
        g.exec = nullptr;
        return fail(c, BC_E_HIP, "bc_render_frame: graph instantiation: %s", hipGetErrorString(ec));
      }
      g.key = key;
    }
    // with a graph only the whole frame is timed (stage slot 1)
    if (ev) {
      if (c->timing_stages) HIPCHECK(c, hipEventRecord(ev[0], st));
      HIPCHECK(c, hipEventRecord(ev[1], st));
    }
    HIPCHECK(c, hipGraphLaunch(g.exec, st));
    if (ev) {
      HIPCHECK(c, hipEventRecord(ev[2], st));
      if (c->timing_stages) HIPCHECK(c, hipEventRecord(ev[3], st));
    }
  }
  HIPCHECK(c, hipEventRecord(c->slot_done[slot], st));
  c->slot_pending[slot] = true;
  HIPCHECK(c, hipEventRecord(c->frame_done, st));
  c->frame_pending = true;
  c->last_learned = c->learned;
  return BC_OK;
}

}  // namespace

extern "C" {

int bc_render_frame(bc_ctx* c, float* out, void* stream) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  return render_impl(c, out, stream, static_cast<float4*>(c->dev[2]), c->max_tiles, false);
}

int bc_render_frame_static(bc_ctx* c, float* out, void* stream) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_render_frame_static: host-only context");
  if (!c->static_sub) return fail(c, BC_E_STATE, "bc_render_frame_static: no static sub-image array on this device");
  if (c->bound && c->has_view && c->view_tiles > BC_STATIC_MAX_TILES)
    return fail(c, BC_E_NOMEM,
                "bc_render_frame_static: the views need up to %lld sub-image tiles, the static array holds %d",
                (long long)c->view_tiles, BC_STATIC_MAX_TILES);
  return render_impl(c, out, stream, c->static_sub, std::min<int64_t>(c->max_tiles, BC_STATIC_MAX_TILES), true);
}

int bc_set_learned(bc_ctx* c, int enable, double coarse_step, double psnr_threshold_db, int validate_stride) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (enable != 0 && enable != 1) return fail(c, BC_E_ARG, "bc_set_learned: enable must be 0 or 1");
  if (!(std::isfinite(coarse_step) && coarse_step > 0.0)) return fail(c, BC_E_ARG, "bc_set_learned: coarse_step must be > 0");
  if (!std::isfinite(psnr_threshold_db)) return fail(c, BC_E_ARG, "bc_set_learned: threshold must be finite");
  if (validate_stride < 1 || validate_stride > 64) return fail(c, BC_E_ARG, "bc_set_learned: validate_stride outside [1, 64]");
  c->learned = enable != 0;
  c->coarse_step = coarse_step;
  c->psnr_threshold = psnr_threshold_db;
  c->val_stride = validate_stride;
  return BC_OK;
}

int bc_set_operator(bc_ctx* c, int op, int step_policy) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (op != BC_OP_COMPOSITE && op != BC_OP_MIP) return fail(c, BC_E_ARG, "bc_set_operator: unknown operator %d", op);
  if (step_policy != BC_STEP_FIXED && step_policy != BC_STEP_PER_VOXEL)
    return fail(c, BC_E_ARG, "bc_set_operator: unknown step policy %d", step_policy);
  if (op == BC_OP_COMPOSITE && step_policy == BC_STEP_PER_VOXEL)
    return fail(c, BC_E_UNSUPPORTED,
                "bc_set_operator: compositing needs one step per frame (its table is opacity-corrected for that step)");
  c->op = op;
  c->step_policy = step_policy;
  return BC_OK;
}

int bc_get_frame_stats(bc_ctx* c, bc_frame_stats* s) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!s) return fail(c, BC_E_ARG, "bc_get_frame_stats: stats is NULL");
  if (!c->frame_pending) return fail(c, BC_E_STATE, "bc_get_frame_stats: no frame rendered");
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  char* meta = static_cast<char*>(c->dev[1]);
  BcCounters h;
  HIPCHECK(c, hipMemcpy(&h, meta + c->off_ctr, offsetof(BcCounters, minmax), hipMemcpyDeviceToHost));
  s->nominal_samples = h.nominal;
  s->evaluated_samples = h.evaluated;
  s->n_tiles = h.total_items;
  s->fell_back = c->last_learned ? (int32_t)h.fallback : -1;
  s->psnr_db = c->last_learned ? h.psnr_db : NAN;
  s->reserved = 0;
  return BC_OK;
}

int bc_set_option(bc_ctx* c, int option, int64_t value) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  switch (option) {
    case BC_OPT_EMPTY_SKIP:
      if (value != 0 && value != 1) return fail(c, BC_E_ARG, "bc_set_option: BC_OPT_EMPTY_SKIP takes 0 or 1");
      c->ess = value != 0;
      return BC_OK;
    case BC_OPT_SAMPLE_CHUNK:
      if (value != 32 && value != 64) return fail(c, BC_E_ARG, "bc_set_option: BC_OPT_SAMPLE_CHUNK takes 32 or 64");
      c->chunk = (int)value;
      return BC_OK;
    case BC_OPT_XCD_QUEUES:
      if (value != 0 && value != 1) return fail(c, BC_E_ARG, "bc_set_option: BC_OPT_XCD_QUEUES takes 0 or 1");
      c->xcd_queues = value != 0;
      return BC_OK;
    case BC_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(c, BC_E_ARG, "bc_set_option: BC_OPT_GRAPH takes 0 or 1");
      if (c->device >= 0) {
        HIPCHECK(c, hipSetDevice(c->device));
        int r = wait_frame(c);
        if (r) return r;
      }
      c->use_graph = value != 0;
      return BC_OK;
    case BC_OPT_TILE_WIDTH: {
      if (value != 4 && value != 8 && value != 16)
        return fail(c, BC_E_ARG, "bc_set_option: BC_OPT_TILE_WIDTH takes 4, 8 or 16");
      const int old = c->tile_shift;
      c->tile_shift = value == 4 ? 2 : (value == 8 ? 3 : 4);
      if (c->planned && c->has_view) {
        int64_t tiles = 0;
        for (const bc_view& v : c->views) tiles += view_tiles_bound(c, v);
        if (tiles > c->max_tiles) {
          c->tile_shift = old;
          return fail(c, BC_E_NOMEM, "bc_set_option: with %lld-pixel-wide tiles the views need %lld sub-image tiles, "
                      "%lld planned", (long long)value, (long long)tiles, (long long)c->max_tiles);
        }
        c->view_tiles = tiles;
      }
      return BC_OK;
    }
    case BC_OPT_RENDER_WORKGROUPS:
      if (value < 1 || value > (1 << 20))
        return fail(c, BC_E_ARG, "bc_set_option: BC_OPT_RENDER_WORKGROUPS outside [1, 2^20]");
      c->render_workgroups = (int)value;
      return BC_OK;
    default:
      return fail(c, BC_E_ARG, "bc_set_option: unknown option %d", option);
  }
}

int bc_autotune(bc_ctx* c, float* out, void* stream, int frames, int64_t chosen[3]) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (frames < 1 || frames > 64) return fail(c, BC_E_ARG, "bc_autotune: frames outside [1, 64]");
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_autotune: host-only context");
  if (c->learned) return fail(c, BC_E_STATE, "bc_autotune: tune with learned frames off");
  if (!c->planned || !c->has_view) return fail(c, BC_E_STATE, "bc_autotune: plan and set the views first");
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  const bool timing = c->timing, graph = c->use_graph;
  const int chunk0 = c->chunk, wgs0 = c->render_workgroups, shift0 = c->tile_shift;
  const int64_t tiles0 = c->view_tiles;
  c->use_graph = false;
  const int shifts[3] = {3, 4, 2};   // 8 x 8, 16 x 4, 4 x 16 screen tiles
  const int chunks[2] = {32, 64};
  const int per_cu[4] = {2, 4, 6, 8};
  double best = 1e300;
  int best_chunk = chunk0, best_wgs = wgs0, best_shift = shift0;
  int64_t best_tiles = tiles0;
  // one untimed frame first: classification and caches
  r = bc_render_frame(c, out, stream);
  for (int si = 0; si < 3 && !r; ++si) {
    c->tile_shift = shifts[si];
    int64_t tiles = 0;
    for (const bc_view& v : c->views) tiles += view_tiles_bound(c, v);
    if (tiles > c->max_tiles) continue;   // this shape does not fit the planned sub-image tiles
    c->view_tiles = tiles;
    for (int ci = 0; ci < 2 && !r; ++ci)
      for (int wi = 0; wi < 4 && !r; ++wi) {
        c->chunk = chunks[ci];
        c->render_workgroups = c->n_cu * per_cu[wi];
        c->timing = true;
        c->timed_frames = 0;
        for (int k = 0; k < frames + 1 && !r; ++k) {
          if (k == 1) c->timed_frames = 0;   // the first frame of a candidate warms it up
          r = bc_render_frame(c, out, stream);
        }
        if (r) break;
        double ms[3];
        int nf = 0;
        r = bc_get_timing(c, ms, &nf);
        if (!r && nf > 0 && ms[1] / nf < best) {
          best = ms[1] / nf;
          best_chunk = c->chunk;
          best_wgs = c->render_workgroups;
          best_shift = c->tile_shift;
          best_tiles = c->view_tiles;
        }
      }
  }
  c->timing = timing;
  c->timed_frames = 0;
  c->use_graph = graph;
  c->chunk = r ? chunk0 : best_chunk;
  c->render_workgroups = r ? wgs0 : best_wgs;
  c->tile_shift = r ? shift0 : best_shift;
  c->view_tiles = r ? tiles0 : best_tiles;
  if (r) return r;
  if (chosen) {
    chosen[0] = best_chunk;
    chosen[1] = best_wgs;
    chosen[2] = 1 << best_shift;
  }
  return BC_OK;
}

int bc_enable_timing(bc_ctx* c, int enable) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_enable_timing: host-only context");
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  if (enable < 0 || enable > 2) return fail(c, BC_E_ARG, "bc_enable_timing: enable must be 0, 1 or 2");
  c->timing = enable != 0;
  c->timing_stages = enable != 2;
  c->timed_frames = 0;
  return BC_OK;
}

int bc_get_timing(bc_ctx* c, double ms_out[3], int* n_frames) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!ms_out) return fail(c, BC_E_ARG, "bc_get_timing: ms_out is NULL");
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_get_timing: host-only context");
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < c->timed_frames; ++k) {
    const hipEvent_t* ev = &c->tev[4 * (size_t)k];
    for (int s = 0; s < 3; ++s) {
      if (!c->timing_stages && s != 1) continue;
      float ms = 0.0f;
      HIPCHECK(c, hipEventElapsedTime(&ms, ev[s], ev[s + 1]));
      acc[s] += ms;
    }
  }
  for (int s = 0; s < 3; ++s) ms_out[s] = acc[s];
  if (n_frames) *n_frames = c->timed_frames;
  return BC_OK;
}

int bc_get_frame_times(bc_ctx* c, double* ms, int cap, int* n_frames) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!ms && cap > 0) return fail(c, BC_E_ARG, "bc_get_frame_times: ms is NULL");
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_get_frame_times: host-only context");
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  const int n = std::min(cap, c->timed_frames);
  for (int k = 0; k < n; ++k) {
    float t = 0.0f;
    const size_t e0 = 4 * (size_t)k + (c->timing_stages ? 0 : 1), e1 = 4 * (size_t)k + (c->timing_stages ? 3 : 2);
    HIPCHECK(c, hipEventElapsedTime(&t, c->tev[e0], c->tev[e1]));
    ms[k] = t;
  }
  if (n_frames) *n_frames = c->timed_frames;
  return BC_OK;
}

int bc_get_bricks(bc_ctx* c, int32_t* lo_hi, float* so, float* mm, int cap, int* n) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!c->planned) return fail(c, BC_E_STATE, "bc_get_bricks: call bc_plan first");
  if (cap < 0) return fail(c, BC_E_ARG, "bc_get_bricks: cap < 0");
  if (n) *n = c->n_bricks;
  const int m = std::min(cap, c->n_bricks);
  for (int b = 0; b < m; ++b) {
    const BcBrick& br = c->bricks[b];
    if (lo_hi)
      for (int a = 0; a < 3; ++a) {
        lo_hi[b * 6 + a] = br.lo[a];
        lo_hi[b * 6 + 3 + a] = br.hi[a];
      }
    if (so) { so[2 * b] = br.scale; so[2 * b + 1] = br.offs; }
    if (mm) { mm[2 * b] = br.vmin; mm[2 * b + 1] = br.vmax; }
  }
  return BC_OK;
}

int bc_get_visibility_order(bc_ctx* c, int view, int32_t* order, int cap) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!order) return fail(c, BC_E_ARG, "bc_get_visibility_order: order is NULL");
  if (!c->frame_pending) return fail(c, BC_E_STATE, "bc_get_visibility_order: no frame rendered");
  if (view < 0 || view >= c->frame_views) return fail(c, BC_E_ARG, "bc_get_visibility_order: bad view %d", view);
  if (cap < c->n_bricks) return fail(c, BC_E_ARG, "bc_get_visibility_order: cap %d < %d bricks", cap, c->n_bricks);
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  char* meta = static_cast<char*>(c->dev[1]);
  HIPCHECK(c, hipMemcpy(order, meta + c->off_order + sizeof(int32_t) * view * c->n_bricks,
                        sizeof(int32_t) * c->n_bricks, hipMemcpyDeviceToHost));
  return BC_OK;
}

int bc_get_rects(bc_ctx* c, int view, int32_t* rects, int cap) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!rects) return fail(c, BC_E_ARG, "bc_get_rects: rects is NULL");
  if (!c->frame_pending) return fail(c, BC_E_STATE, "bc_get_rects: no frame rendered");
  if (view < 0 || view >= c->frame_views) return fail(c, BC_E_ARG, "bc_get_rects: bad view %d", view);
  if (cap < c->n_bricks) return fail(c, BC_E_ARG, "bc_get_rects: cap %d < %d bricks", cap, c->n_bricks);
  HIPCHECK(c, hipSetDevice(c->device));
  int r = wait_frame(c);
  if (r) return r;
  char* meta = static_cast<char*>(c->dev[1]);
  HIPCHECK(c, hipMemcpy(rects, meta + c->off_rects + sizeof(int32_t) * 4 * view * c->n_bricks,
                        sizeof(int32_t) * 4 * c->n_bricks, hipMemcpyDeviceToHost));
  for (int b = 0; b < c->n_bricks; ++b)
    for (int k = 0; k < 4; ++k) rects[4 * b + k] *= (k & 1) ? (64 >> c->frame_tile_shift) : (1 << c->frame_tile_shift);
  return BC_OK;
}

int bc_read_brick(bc_ctx* c, int b, void* dst, size_t cap, int32_t dims[3]) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!c->loaded) return fail(c, BC_E_STATE, "bc_read_brick: bricks not loaded");
  if (b < 0 || b >= c->n_bricks) return fail(c, BC_E_ARG, "bc_read_brick: brick %d out of range", b);
  const BcBrick& br = c->bricks[b];
  const size_t bytes = (size_t)br.mb[0] * br.mb[1] * br.mb[2] * BC_MB_ELEMS * c->elem_bytes;
  if (dims)
    for (int a = 0; a < 3; ++a) dims[a] = br.gdim[a];
  if (!dst) return BC_OK;
  if (cap < bytes) return fail(c, BC_E_ARG, "bc_read_brick: need %zu bytes", bytes);
  HIPCHECK(c, hipSetDevice(c->device));
  (void)wait_frame(c);
  HIPCHECK(c, hipMemcpy(dst, static_cast<char*>(c->dev[0]) + br.offset * c->elem_bytes, bytes, hipMemcpyDeviceToHost));
  return BC_OK;
}

}  // extern "C"

// ======================================================================
// Learned upsampler
// ======================================================================
namespace {

CnnPackTable cnn_pack_table(bc_ctx* c, const CnnLayout& L) {
  CnnPackTable t;
  auto ent = [&](size_t off, int w_off, int cin, int cout, int ks, int nt, int tr) {
    CnnPackEntry e;
    e.dst = reinterpret_cast<uint16_t*>(c->cnn_ws + off);
    e.w_off = w_off; e.cin = cin; e.cout = cout; e.ks = ks; e.nt = nt; e.transposed = tr;
    return e;
  };
  t.e[0] = ent(L.f1, CNN_OFF_W1, 4, 32, 2, 2, 0);
  t.e[1] = ent(L.f2, CNN_OFF_W2, 32, 32, 9, 2, 0);
  t.e[2] = ent(L.f3, CNN_OFF_W3, 32, 16, 9, 1, 0);
  t.e[3] = ent(L.b3, CNN_OFF_W3, 32, 16, 5, 2, 1);
  t.e[4] = ent(L.b2, CNN_OFF_W2, 32, 32, 9, 2, 1);
  t.n = 5;
  return t;
}

int cnn_check_images(bc_ctx* c, const char* who, int n, int h, int w) {
  if (!c->cnn_bound) return fail(c, BC_E_STATE, "%s: bind the upsampler workspace first", who);
  if (!c->cnn_has_w) return fail(c, BC_E_STATE, "%s: set the upsampler weights first", who);
  if (n < 1 || h < 1 || w < 1 || n > c->cnn_max_n || h > c->cnn_max_h || w > c->cnn_max_w)
    return fail(c, BC_E_ARG, "%s: %d images of %d x %d exceed the planned %d of %d x %d", who, n, w, h, c->cnn_max_n,
                c->cnn_max_w, c->cnn_max_h);
  return BC_OK;
}

// forward + loss + backward into the gradient vector (no update)
int cnn_gradients(bc_ctx* c, const float* coarse, const float* target, int n, int h, int w, hipStream_t st) {
  const CnnLayout L = cnn_layout(n, h, w);
  char* ws = c->cnn_ws;
  auto U16 = [&](size_t off) { return reinterpret_cast<uint16_t*>(ws + off); };
  auto F32 = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
  auto FR = [&](size_t off) { return reinterpret_cast<const uint4*>(ws + off); };
  const float* wts = F32(L.w);
  CnnLayerArgs a{};
  a.h = h; a.w = w;
  // forward
  a.img = coarse; a.in = nullptr; a.out = U16(L.a1); a.bias = wts + CNN_OFF_B1; a.wf = FR(L.f1);
  HIPCHECK(c, cnn_launch_layer(1, 0, a, n, st));
  a.img = nullptr; a.in = U16(L.a1); a.out = U16(L.a2); a.bias = wts + CNN_OFF_B2; a.wf = FR(L.f2);
  HIPCHECK(c, cnn_launch_layer(2, 0, a, n, st));
  a.img = coarse; a.in = U16(L.a2); a.out = U16(L.gy); a.bias = wts + CNN_OFF_B3; a.wf = FR(L.f3);
  a.target = target; a.loss_part = F32(L.loss);
  a.grad_scale = (float)(2.0 / ((double)n * 4.0 * h * w * 4.0));
  HIPCHECK(c, cnn_launch_layer(3, 2, a, n, st));
  // backward-data through layers 3 and 2 (ReLU masks from a2 and a1)
  CnnLayerArgs bd{};
  bd.h = h; bd.w = w;
  bd.in = U16(L.gy); bd.out = U16(L.gz2); bd.mask = U16(L.a2); bd.wf = FR(L.b3);
  HIPCHECK(c, cnn_launch_layer(3, 1, bd, n, st));
  bd.in = U16(L.gz2); bd.out = U16(L.gz1); bd.mask = U16(L.a1); bd.wf = FR(L.b2);
  HIPCHECK(c, cnn_launch_layer(2, 1, bd, n, st));
  // backward-weights per layer, then deterministic reductions
  float* g = F32(L.g);
  struct { int layer, cin, cout; const float* img; const uint16_t* x; const uint16_t* gr; int w_off, b_off; } jobs[3] = {
      {3, 32, 16, nullptr, U16(L.a2), U16(L.gy), CNN_OFF_W3, CNN_OFF_B3},
      {2, 32, 32, nullptr, U16(L.a1), U16(L.gz2), CNN_OFF_W2, CNN_OFF_B2},
      {1, 4, 32, coarse, nullptr, U16(L.gz1), CNN_OFF_W1, CNN_OFF_B1}};
  for (auto& j : jobs) {
    CnnWgradArgs wa{};
    wa.img = j.img; wa.x = j.x; wa.g = j.gr; wa.part = F32(L.part); wa.h = h; wa.w = w;
    HIPCHECK(c, cnn_launch_wgrad(j.layer, wa, n, st));
    const int nw = j.cout * j.cin * 9;
    HIPCHECK(c, cnn_launch_reduce(F32(L.part), L.tiles, nw + j.cout, g + j.w_off, g + j.b_off, nw, st));
  }
  return BC_OK;
}

int cnn_infer(bc_ctx* c, const CnnLayout& L, const float* coarse, float* fine, int n, int h, int w, hipStream_t st) {
  CnnInferArgs a;
  a.x = coarse;
  a.out = fine;
  a.params = reinterpret_cast<const float*>(c->cnn_ws + L.w);
  a.wf1 = reinterpret_cast<const uint4*>(c->cnn_ws + L.f1);
  a.wf2 = reinterpret_cast<const uint4*>(c->cnn_ws + L.f2);
  a.wf3 = reinterpret_cast<const uint4*>(c->cnn_ws + L.f3);
  a.h = h;
  a.w = w;
  HIPCHECK(c, cnn_launch_infer(a, n, st));
  return BC_OK;
}

int cnn_read_loss(bc_ctx* c, int n, int h, int w, float* loss, hipStream_t st) {
  const CnnLayout L = cnn_layout(n, h, w);
  c->cnn_loss_host.resize((size_t)L.tiles);
  HIPCHECK(c, hipMemcpyAsync(c->cnn_loss_host.data(), c->cnn_ws + L.loss, sizeof(float) * L.tiles,
                             hipMemcpyDeviceToHost, st));
  HIPCHECK(c, hipStreamSynchronize(st));
  double s = 0.0;
  for (float v : c->cnn_loss_host) s += v;
  *loss = (float)(s / ((double)n * 4.0 * h * w * 4.0));
  return BC_OK;
}

}  // namespace

extern "C" {

int bc_cnn_plan(bc_ctx* c, int max_n, int max_h, int max_w, size_t* bytes) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!bytes) return fail(c, BC_E_ARG, "bc_cnn_plan: bytes is NULL");
  if (max_n < 1 || max_n > 64 || max_h < 1 || max_w < 1 || max_h > 8192 || max_w > 8192)
    return fail(c, BC_E_ARG, "bc_cnn_plan: need 1 <= max_n <= 64 and coarse size in [1, 8192]");
  if (c->cnn_bound) return fail(c, BC_E_STATE, "bc_cnn_plan: workspace already bound");
  const CnnLayout L = cnn_layout(max_n, max_h, max_w);
  c->cnn_max_n = max_n;
  c->cnn_max_h = max_h;
  c->cnn_max_w = max_w;
  c->cnn_bytes = L.total;
  c->cnn_planned = true;
  *bytes = L.total;
  return BC_OK;
}

int bc_cnn_bind(bc_ctx* c, void* ws, size_t bytes) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (c->device < 0) return fail(c, BC_E_STATE, "bc_cnn_bind: host-only context");
  if (!c->cnn_planned) return fail(c, BC_E_STATE, "bc_cnn_bind: call bc_cnn_plan first");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(c, BC_E_ARG, "bc_cnn_bind: workspace NULL or not 256-byte aligned");
  if (bytes < c->cnn_bytes) return fail(c, BC_E_NOMEM, "bc_cnn_bind: %zu bytes, %zu planned", bytes, c->cnn_bytes);
  c->cnn_ws = static_cast<char*>(ws);
  c->cnn_bound = true;
  c->cnn_has_w = false;
  return BC_OK;
}

int bc_cnn_set_weights(bc_ctx* c, const float* w, const float* adam_m, const float* adam_v, size_t n, int64_t step) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!c->cnn_bound) return fail(c, BC_E_STATE, "bc_cnn_set_weights: bind the workspace first");
  if (!w) return fail(c, BC_E_ARG, "bc_cnn_set_weights: w is NULL");
  if (n != CNN_N_PARAMS) return fail(c, BC_E_ARG, "bc_cnn_set_weights: n = %zu, the network has %d parameters", n, CNN_N_PARAMS);
  if ((adam_m == nullptr) != (adam_v == nullptr)) return fail(c, BC_E_ARG, "bc_cnn_set_weights: give both Adam moments or neither");
  if (step < 0) return fail(c, BC_E_ARG, "bc_cnn_set_weights: step < 0");
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(w[i])) return fail(c, BC_E_ARG, "bc_cnn_set_weights: parameter %zu is not finite", i);
  HIPCHECK(c, hipSetDevice(c->device));
  (void)wait_frame(c);
  const CnnLayout L = cnn_layout(c->cnn_max_n, c->cnn_max_h, c->cnn_max_w);
  const size_t b = sizeof(float) * CNN_N_PARAMS;
  HIPCHECK(c, hipMemcpy(c->cnn_ws + L.w, w, b, hipMemcpyHostToDevice));
  if (adam_m) {
    HIPCHECK(c, hipMemcpy(c->cnn_ws + L.m, adam_m, b, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->cnn_ws + L.v, adam_v, b, hipMemcpyHostToDevice));
  } else {
    std::vector<float> z(CNN_N_PARAMS, 0.0f);
    HIPCHECK(c, hipMemcpy(c->cnn_ws + L.m, z.data(), b, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->cnn_ws + L.v, z.data(), b, hipMemcpyHostToDevice));
  }
  HIPCHECK(c, cnn_launch_pack(reinterpret_cast<const float*>(c->cnn_ws + L.w), cnn_pack_table(c, L), nullptr));
  HIPCHECK(c, hipStreamSynchronize(nullptr));
  c->cnn_step = step;
  c->cnn_has_w = true;
  return BC_OK;
}

int bc_cnn_get_weights(bc_ctx* c, float* w, float* adam_m, float* adam_v, size_t n, int64_t* step) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!c->cnn_has_w) return fail(c, BC_E_STATE, "bc_cnn_get_weights: no weights set");
  if (n != CNN_N_PARAMS) return fail(c, BC_E_ARG, "bc_cnn_get_weights: n = %zu, the network has %d parameters", n, CNN_N_PARAMS);
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipDeviceSynchronize());
  const CnnLayout L = cnn_layout(c->cnn_max_n, c->cnn_max_h, c->cnn_max_w);
  const size_t b = sizeof(float) * CNN_N_PARAMS;
  if (w) HIPCHECK(c, hipMemcpy(w, c->cnn_ws + L.w, b, hipMemcpyDeviceToHost));
  if (adam_m) HIPCHECK(c, hipMemcpy(adam_m, c->cnn_ws + L.m, b, hipMemcpyDeviceToHost));
  if (adam_v) HIPCHECK(c, hipMemcpy(adam_v, c->cnn_ws + L.v, b, hipMemcpyDeviceToHost));
  if (step) *step = c->cnn_step;
  return BC_OK;
}

int bc_cnn_forward(bc_ctx* c, const float* coarse, float* fine, int n, int h, int w, void* stream) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!coarse || !fine) return fail(c, BC_E_ARG, "bc_cnn_forward: null image");
  if ((reinterpret_cast<uintptr_t>(coarse) | reinterpret_cast<uintptr_t>(fine)) & 15)
    return fail(c, BC_E_ARG, "bc_cnn_forward: images must be 16-byte aligned");
  int r = cnn_check_images(c, "bc_cnn_forward", n, h, w);
  if (r) return r;
  HIPCHECK(c, hipSetDevice(c->device));
  const CnnLayout L = cnn_layout(c->cnn_max_n, c->cnn_max_h, c->cnn_max_w);
  return cnn_infer(c, L, coarse, fine, n, h, w, static_cast<hipStream_t>(stream));
}

int bc_cnn_gradients(bc_ctx* c, const float* coarse, const float* target, int n, int h, int w, float* grad,
                     float* loss) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!coarse || !target) return fail(c, BC_E_ARG, "bc_cnn_gradients: null image");
  int r = cnn_check_images(c, "bc_cnn_gradients", n, h, w);
  if (r) return r;
  HIPCHECK(c, hipSetDevice(c->device));
  // the per-layer buffers are laid out for the size of this call
  r = cnn_gradients(c, coarse, target, n, h, w, nullptr);
  if (r) return r;
  const CnnLayout L = cnn_layout(n, h, w);
  if (grad) HIPCHECK(c, hipMemcpy(grad, c->cnn_ws + L.g, sizeof(float) * CNN_N_PARAMS, hipMemcpyDeviceToHost));
  if (loss) return cnn_read_loss(c, n, h, w, loss, nullptr);
  HIPCHECK(c, hipStreamSynchronize(nullptr));
  return BC_OK;
}

int bc_cnn_train_step(bc_ctx* c, const float* coarse, const float* target, int n, int h, int w, float lr,
                      float* loss, void* stream) {
  if (!c) return BC_E_ARG;
  c->err.clear();
  if (!coarse || !target) return fail(c, BC_E_ARG, "bc_cnn_train_step: null image");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(c, BC_E_ARG, "bc_cnn_train_step: lr must be finite and > 0");
  int r = cnn_check_images(c, "bc_cnn_train_step", n, h, w);
  if (r) return r;
  HIPCHECK(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  r = cnn_gradients(c, coarse, target, n, h, w, st);
  if (r) return r;
  const CnnLayout Lg = cnn_layout(n, h, w);
  const CnnLayout L = cnn_layout(c->cnn_max_n, c->cnn_max_h, c->cnn_max_w);
  float* wv = reinterpret_cast<float*>(c->cnn_ws + L.w);
  c->cnn_step += 1;
  HIPCHECK(c, cnn_launch_adam(wv, reinterpret_cast<float*>(c->cnn_ws + L.m), reinterpret_cast<float*>(c->cnn_ws + L.v),
                              reinterpret_cast<const float*>(c->cnn_ws + Lg.g), CNN_N_PARAMS, lr, c->cnn_step, st));
  HIPCHECK(c, cnn_launch_pack(wv, cnn_pack_table(c, L), st));
  if (loss) return cnn_read_loss(c, n, h, w, loss, st);
  return BC_OK;
}

}  // extern "C"
