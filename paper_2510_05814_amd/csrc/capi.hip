// The C ABI of include/smoe.h: host-side validation, workspace layout and the launch
// sequences of each call.  No device memory is allocated here.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "smoe_internal.h"

using namespace smoe;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool valid_shape(int32_t K, int32_t C, int32_t order) {
  if (K < 0 || (C != 1 && C != 3) || (order != 0 && order != 1)) return false;
  // every [K][NP] and pair index fits in int32 arithmetic
  return (long long)K * 16 < (1LL << 31);
}

bool valid_model(const smoe_model* m) {
  return m && valid_shape(m->K, m->C, m->order) && (m->K == 0 || m->params);
}

bool valid_raster(int32_t W, int32_t H, int32_t scale, int32_t ox, int32_t oy) {
  if (W < 1 || H < 1 || W > 65536 || H > 65536) return false;
  if (scale < 1 || scale > 64) return false;
  return std::abs(ox) <= (1 << 22) && std::abs(oy) <= (1 << 22);
}

// Truncation radius in [2^-30, 2^30]: the ellipse bound r^2 is then a normal binary32 number
// whose compare-free cut constants are exact.
bool valid_radius(float r) { return r >= 0x1p-30f && r <= 0x1p30f; }
// Sharpening factor: 0 (none) or a finite positive bandwidth divisor.
bool valid_sharpen(float f) { return f == 0.0f || (f > 0.0f && std::isfinite(f)); }
bool no_sharpen(float f) { return f == 0.0f || f == 1.0f; }
bool valid_box(int32_t b) { return b == SMOE_BOX_SQUARE || b == SMOE_BOX_TIGHT; }
bool valid_mode(int32_t m) { return m == SMOE_MODE_SMOE || m == SMOE_MODE_RBF; }
bool valid_trunc(int32_t t) { return t == SMOE_TRUNC_RENDER || t == SMOE_TRUNC_GRADIENT; }

// The render's bound in its compare-free form (Segs::cut_scale, cut_offset).  With the ellipse
// test in the render: q <= r^2, scale 2^k with r^2 2^k in [2^60, 2^61) (the radius range keeps
// r^2 a normal binary32 number with a representable power-of-two scale).  With the block
// lists deciding the render: the term's exponent a >= -125, as min(a, fma(a, 2^60, 125 2^60)).
void set_render_bound(Segs& S) {
  if (S.trunc == SMOE_TRUNC_RENDER) {
    S.r2_render = S.r * S.r;
    int e = 0;
    std::frexp(S.r2_render, &e);  // r2_render = f 2^e with f in [0.5, 1)
    S.cut_scale = std::ldexp(1.0f, 61 - e);
    S.cut_offset = -S.r2_render * S.cut_scale;
  } else {
    S.r2_render = 0.0f;  // no bound on q
    S.cut_scale = 0x1p60f;
    S.cut_offset = 125.0f * 0x1p60f;
  }
}

// Blocks of a raster: the 16x16 blocks of its scale's output grid (aligned to multiples of
// 16 in the output coordinate) that its pixels touch.
long long raster_tiles(int32_t W, int32_t H, int32_t ox, int32_t oy) {
  return (long long)blocks_across(W, ox) * blocks_across(H, oy);
}

// The single raster of a non-batched call as a one-segment Segs.
bool single_segs(const smoe_model* m, const smoe_grid* g, Segs* out) {
  if (!valid_model(m) || !g ||
      !valid_raster(g->width, g->height, g->scale, g->origin_x, g->origin_y) ||
      !valid_radius(g->radius) || !valid_sharpen(g->sharpen) || !valid_box(g->box) ||
      !valid_mode(g->mode) || !valid_trunc(g->trunc))
    return false;
  Segs S;
  std::memset(&S, 0, sizeof(S));
  smoe_segment& o = S.one;
  o.width = g->width;
  o.height = g->height;
  o.scale = g->scale;
  o.origin_x = g->origin_x;
  o.origin_y = g->origin_y;
  o.sharpen = g->sharpen;
  o.num_kernels = m->K;
  S.r = g->radius;
  S.r2 = g->radius * g->radius;
  S.box = g->box;
  S.mode = g->mode;
  S.trunc = g->trunc;
  set_render_bound(S);
  S.T = (int)raster_tiles(g->width, g->height, g->origin_x, g->origin_y);
  S.K = m->K;
  *out = S;
  return true;
}

// Checks a host segment table (rasters valid, offsets equal to their running sums, model
// rows inside [0, rows)) and returns its totals.
bool check_segments(const smoe_segment* h, int32_t n, int32_t rows, int* T, int* K) {
  if (!h || n < 1) return false;
  long long t = 0, k = 0, px = 0;
  for (int i = 0; i < n; ++i) {
    const smoe_segment& s = h[i];
    if (!valid_raster(s.width, s.height, s.scale, s.origin_x, s.origin_y) ||
        !valid_sharpen(s.sharpen))
      return false;
    if (s.num_kernels < 0 || s.param_offset < 0) return false;
    if ((long long)s.param_offset + s.num_kernels > rows) return false;
    if (s.kernel_offset != k || s.tile_offset != t || s.pixel_offset != px) return false;
    k += s.num_kernels;
    t += raster_tiles(s.width, s.height, s.origin_x, s.origin_y);
    px += (long long)s.width * s.height;
  }
  if (t >= (1LL << 31) || k * 16 >= (1LL << 31)) return false;
  *T = (int)t;
  *K = (int)k;
  return true;
}

bool batch_segs(const smoe_batch* b, Segs* out) {
  if (!b || !valid_shape(0, b->C, b->order) || !b->params || !b->segments ||
      b->num_params_rows < 0 || !valid_radius(b->radius) || !valid_box(b->box) ||
      !valid_mode(b->mode) || !valid_trunc(b->trunc))
    return false;
  Segs S;
  std::memset(&S, 0, sizeof(S));
  if (!check_segments(b->segments_host, b->num_segments, b->num_params_rows, &S.T, &S.K))
    return false;
  S.tab = b->segments;
  S.n = b->num_segments;
  S.r = b->radius;
  S.r2 = b->radius * b->radius;
  S.box = b->box;
  S.mode = b->mode;
  S.trunc = b->trunc;
  set_render_bound(S);
  *out = S;
  return true;
}

bool bins_match(const smoe_bins* b, int K, int C, int order) {
  return b && b->K == K && b->C == C && b->order == order && b->status && b->ranges && b->vals &&
         b->records && b->tile_rects && b->native_rects;
}

struct Layout {
  size_t tile_rects, native_rects, counts, records, tile_counts, ranges, keys, vals, vals_alt,
      pair_grads, tile_loss, status, total;
};

// grads = false: a render-only workspace, without the per-pair gradient partials.
Layout layout_of(int32_t K, int32_t C, int32_t order, int32_t max_tiles, int32_t capacity,
                 bool grads = true) {
  const size_t rs = (size_t)record_stride(C, order);
  const size_t np = (size_t)num_params(C, order);
  Layout L;
  size_t o = 0;
  L.tile_rects = o; o = align_up(o + (size_t)K * 4 * sizeof(int32_t));
  L.native_rects = o; o = align_up(o + (size_t)K * 4 * sizeof(int32_t));
  L.counts = o;     o = align_up(o + (size_t)K * sizeof(int32_t));
  L.records = o;    o = align_up(o + (size_t)K * rs * sizeof(float));
  L.tile_counts = o; o = align_up(o + (size_t)max_tiles * sizeof(int32_t));
  L.ranges = o;     o = align_up(o + (size_t)max_tiles * 2 * sizeof(int32_t));
  L.keys = o;       o = align_up(o + (size_t)capacity * sizeof(uint32_t));
  L.vals = o;       o = align_up(o + (size_t)capacity * sizeof(uint32_t));
  L.vals_alt = o;   o = align_up(o + (size_t)capacity * sizeof(uint32_t));
  // partial rows: kSlots per kernel (the fit step's kernel-major rows), then one per pair
  L.pair_grads = o;
  o = align_up(o + (grads ? ((size_t)K * kSlots + (size_t)capacity) * partial_stride((int)np) *
                                sizeof(float)
                          : 0));
  L.tile_loss = o;  o = align_up(o + (size_t)max_tiles * sizeof(float));
  L.status = o;     o = align_up(o + 8 * sizeof(int32_t));
  L.total = o;
  return L;
}

// The HIP error behind the last SMOE_ERR_HIP of this thread, for smoe_last_error().
thread_local char g_last_error[256] = "no error";

inline smoe_status hip_status(hipError_t e) {
  if (e == hipSuccess) return SMOE_OK;
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", hipGetErrorName(e),
                hipGetErrorString(e));
  return SMOE_ERR_HIP;
}

// hipGetLastError() reports the last failure of any HIP call on the thread, including
// calls made by other code before ours; a launching entry point clears it first so that
// the status it returns is about its own launches only.
inline void clear_stale_error() { (void)hipGetLastError(); }

// The rasters of a fit state: its segment table (batched fit) or its single grid.
bool fit_segs(const smoe_fit_state* st, Segs* S) {
  if (st->num_segments > 0) {
    if (!st->segments || !st->segments_host || !valid_radius(st->grid.radius) ||
        !valid_box(st->grid.box) || !valid_mode(st->grid.mode) || !valid_trunc(st->grid.trunc))
      return false;
    std::memset(S, 0, sizeof(*S));
    if (!check_segments(st->segments_host, st->num_segments, st->K, &S->T, &S->K)) return false;
    for (int i = 0; i < st->num_segments; ++i) {
      const smoe_segment& s = st->segments_host[i];
      if (s.scale != 1 || s.origin_x != 0 || s.origin_y != 0 ||
          s.param_offset != s.kernel_offset || !no_sharpen(s.sharpen))
        return false;
    }
    if (S->K != st->K) return false;
    S->tab = st->segments;
    S->n = st->num_segments;
    S->r = st->grid.radius;
    S->r2 = st->grid.radius * st->grid.radius;
    S->box = st->grid.box;
    S->mode = st->grid.mode;
    S->trunc = st->grid.trunc;
    set_render_bound(*S);
    return true;
  }
  const smoe_model m{st->K, st->C, st->order, st->model};
  if (!single_segs(&m, &st->grid, S)) return false;
  return st->grid.scale == 1 && st->grid.origin_x == 0 && st->grid.origin_y == 0 &&
         no_sharpen(st->grid.sharpen);
}

smoe_status fit_step(smoe_fit_state* st, const float* target, float* loss_out,
                     void* const* ev, void* stream) {
  clear_stale_error();
  if (!st || !target) return SMOE_ERR_INVALID;
  Segs S;
  if (!valid_shape(st->K, st->C, st->order) || (st->K > 0 && !st->model) || !fit_segs(st, &S) ||
      !bins_match(&st->bins, S.K, st->C, st->order))
    return SMOE_ERR_INVALID;
  if (!st->raw || !st->adam_m || !st->adam_v || !st->image || !st->denom || !st->step ||
      !st->scalars || !st->bins.pair_grads || !st->bins.tile_loss ||
      st->max_steps < 0)
    return SMOE_ERR_INVALID;
  if (S.T > st->bins.max_tiles) return SMOE_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto mark = [&](int i) -> hipError_t {
    return (ev && ev[i]) ? hipEventRecord(static_cast<hipEvent_t>(ev[i]), s) : hipSuccess;
  };
  // The pair storage as fixed-width block buckets: block t owns entries [t W, t W + W).  An
  // entry is (kernel id << shift) | low with low < kSlots + W <= 2^shift (the row of its
  // partial, k_scatter_fixed), so the kernel ids must fit in 32 - shift bits.
  const int width = st->bins.capacity / S.T;
  int shift = 0;
  while ((1LL << shift) < (long long)width + kSlots) ++shift;
  if (((long long)S.K << shift) > (1LL << 32)) return SMOE_ERR_TOO_LARGE;
  hipError_t e = mark(0);
  if (e == hipSuccess && !st->prepared)
    e = launch_prepare_fit(st->C, st->order, st->model, S, st->bins, s);
  if (e == hipSuccess)
    e = launch_scatter_fixed(S, st->bins, st->model, num_params(st->C, st->order), width, shift,
                             st->step, st->adam, st->scalars, s);
  if (e == hipSuccess) e = mark(1);
  if (e == hipSuccess) e = launch_fit_tile(*st, S, width, shift, target, s);
  if (e == hipSuccess) e = mark(2);
  if (e == hipSuccess) e = launch_adam_fit(*st, S, shift, loss_out, s);
  if (e == hipSuccess) e = mark(3);
  if (e == hipSuccess) st->prepared = 1;
  return hip_status(e);
}

// Static workspace of smoe_render_noalloc: a file-scope device array (one copy per GPU,
// held until the process ends).  In host code `scratch` names a host-side stand-in; the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed to kernels.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (nullptr and a HIP error if it
// cannot be had).
hipError_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// The largest pair capacity whose render-only layout fits the static workspace (-1: the
// per-kernel and per-block arrays alone do not fit).
long long static_capacity(int32_t K, int32_t C, int32_t order, int32_t T) {
  const size_t fixed = layout_of(K, C, order, T, 0, false).total;
  if (fixed > kStaticScratchBytes) return -1;
  // three u32 arrays per pair (keys, vals, vals_alt), each aligned up once
  long long cap = (long long)((kStaticScratchBytes - fixed - 3 * kAlign) / (3 * sizeof(uint32_t)));
  cap = std::min(cap, (long long)INT32_MAX / 16);
  while (cap > 0 && layout_of(K, C, order, T, (int32_t)cap, false).total > kStaticScratchBytes)
    cap -= 64;
  return cap;
}

}  // namespace

extern "C" {

int32_t smoe_version(void) { return 100; }

const char* smoe_last_error(void) { return g_last_error; }

size_t smoe_bins_workspace_bytes(int32_t K, int32_t C, int32_t order, int32_t max_tiles,
                                 int32_t capacity) {
  if (!valid_shape(K, C, order) || max_tiles < 1 || capacity < 0) return 0;
  return layout_of(K, C, order, max_tiles, capacity).total;
}

namespace {

smoe_status layout_into(smoe_bins* out, void* workspace, size_t bytes, int32_t K, int32_t C,
                        int32_t order, int32_t max_tiles, int32_t capacity, bool grads) {
  if (!out || !workspace || !valid_shape(K, C, order) || max_tiles < 1 || capacity < 0)
    return SMOE_ERR_INVALID;
  if (((uintptr_t)workspace & (kAlign - 1)) != 0) return SMOE_ERR_INVALID;
  const Layout L = layout_of(K, C, order, max_tiles, capacity, grads);
  if (bytes < L.total) return SMOE_ERR_INVALID;
  char* base = static_cast<char*>(workspace);
  smoe_bins b;
  std::memset(&b, 0, sizeof(b));
  b.K = K;
  b.C = C;
  b.order = order;
  b.max_tiles = max_tiles;
  b.capacity = capacity;
  b.tile_rects = reinterpret_cast<int32_t*>(base + L.tile_rects);
  b.native_rects = reinterpret_cast<int32_t*>(base + L.native_rects);
  b.counts = reinterpret_cast<int32_t*>(base + L.counts);
  b.records = reinterpret_cast<float*>(base + L.records);
  b.record_stride = record_stride(C, order);
  b.tile_counts = reinterpret_cast<int32_t*>(base + L.tile_counts);
  b.ranges = reinterpret_cast<int32_t*>(base + L.ranges);
  b.keys = reinterpret_cast<uint32_t*>(base + L.keys);
  b.vals = reinterpret_cast<uint32_t*>(base + L.vals);
  b.vals_alt = reinterpret_cast<uint32_t*>(base + L.vals_alt);
  b.pair_grads = grads ? reinterpret_cast<float*>(base + L.pair_grads) : nullptr;
  b.tile_loss = reinterpret_cast<float*>(base + L.tile_loss);
  b.status = reinterpret_cast<int32_t*>(base + L.status);
  *out = b;
  return SMOE_OK;
}

}  // namespace

smoe_status smoe_bins_layout(smoe_bins* out, void* workspace, size_t bytes, int32_t K, int32_t C,
                             int32_t order, int32_t max_tiles, int32_t capacity) {
  return layout_into(out, workspace, bytes, K, C, order, max_tiles, capacity, true);
}

size_t smoe_render_workspace_bytes(int32_t K, int32_t C, int32_t order, int32_t max_tiles,
                                   int32_t capacity) {
  if (!valid_shape(K, C, order) || max_tiles < 1 || capacity < 0) return 0;
  return layout_of(K, C, order, max_tiles, capacity, false).total;
}

smoe_status smoe_render_workspace_layout(smoe_bins* out, void* workspace, size_t bytes, int32_t K,
                                         int32_t C, int32_t order, int32_t max_tiles,
                                         int32_t capacity) {
  return layout_into(out, workspace, bytes, K, C, order, max_tiles, capacity, false);
}

smoe_status smoe_segments_layout(smoe_segment* segs, int32_t n, int32_t* total_kernels,
                                 int32_t* total_tiles, int64_t* total_pixels) {
  if (!segs || n < 1) return SMOE_ERR_INVALID;
  long long t = 0, k = 0, px = 0;
  for (int i = 0; i < n; ++i) {
    smoe_segment& s = segs[i];
    if (!valid_raster(s.width, s.height, s.scale, s.origin_x, s.origin_y) || s.num_kernels < 0 ||
        s.param_offset < 0 || !valid_sharpen(s.sharpen))
      return SMOE_ERR_INVALID;
    s.kernel_offset = (int32_t)k;
    s.tile_offset = (int32_t)t;
    s.pixel_offset = px;
    k += s.num_kernels;
    t += raster_tiles(s.width, s.height, s.origin_x, s.origin_y);
    px += (long long)s.width * s.height;
    if (t >= (1LL << 31) || k * 16 >= (1LL << 31)) return SMOE_ERR_INVALID;
  }
  if (total_kernels) *total_kernels = (int32_t)k;
  if (total_tiles) *total_tiles = (int32_t)t;
  if (total_pixels) *total_pixels = px;
  return SMOE_OK;
}

smoe_status smoe_bin(const smoe_model* model, const smoe_grid* grid, smoe_bins* bins,
                     void* stream) {
  clear_stale_error();
  Segs S;
  if (!single_segs(model, grid, &S) || !bins_match(bins, model->K, model->C, model->order))
    return SMOE_ERR_INVALID;
  if (S.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  return hip_status(launch_bin(model->C, model->order, model->params, S, *bins,
                               static_cast<hipStream_t>(stream)));
}

smoe_status smoe_render(const smoe_model* model, const smoe_grid* grid, const smoe_bins* bins,
                        float* image, float* denom, const float* target, float* loss_out,
                        void* stream) {
  clear_stale_error();
  Segs S;
  if (!single_segs(model, grid, &S) || !bins_match(bins, model->K, model->C, model->order) ||
      !image)
    return SMOE_ERR_INVALID;
  if (S.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  const bool loss = target && loss_out;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e =
      launch_render(model->C, model->order, S, *bins, image, denom, loss ? target : nullptr, s);
  if (e == hipSuccess && loss) {
    const float inv_n = (float)(1.0 / ((double)grid->width * grid->height * model->C));
    e = launch_loss_reduce(*bins, S.T, inv_n, loss_out, s);
  }
  return hip_status(e);
}

smoe_status smoe_render_backward(const smoe_model* model, const smoe_grid* grid,
                                 const smoe_bins* bins, const float* image, const float* denom,
                                 const float* grad_image, const float* target, float* grads,
                                 void* stream) {
  clear_stale_error();
  Segs S;
  if (!single_segs(model, grid, &S) || !bins_match(bins, model->K, model->C, model->order) ||
      !image || !denom || !grads || (grad_image == nullptr) == (target == nullptr) ||
      !bins->pair_grads || !no_sharpen(grid->sharpen))
    return SMOE_ERR_INVALID;
  if (S.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e =
      launch_backward(model->C, model->order, S, *bins, image, denom, grad_image, target, s);
  if (e == hipSuccess) e = launch_gather(model->C, model->order, S, *bins, grads, s);
  return hip_status(e);
}

smoe_status smoe_bin_batched(const smoe_batch* batch, smoe_bins* bins, void* stream) {
  clear_stale_error();
  Segs S;
  if (!batch_segs(batch, &S) || !bins_match(bins, S.K, batch->C, batch->order))
    return SMOE_ERR_INVALID;
  if (S.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  return hip_status(launch_bin(batch->C, batch->order, batch->params, S, *bins,
                               static_cast<hipStream_t>(stream)));
}

smoe_status smoe_render_batched(const smoe_batch* batch, const smoe_bins* bins, float* images,
                                float* denoms, void* stream) {
  clear_stale_error();
  Segs S;
  if (!batch_segs(batch, &S) || !bins_match(bins, S.K, batch->C, batch->order) || !images)
    return SMOE_ERR_INVALID;
  if (S.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  return hip_status(launch_render(batch->C, batch->order, S, *bins, images, denoms, nullptr,
                                  static_cast<hipStream_t>(stream)));
}

smoe_status smoe_render_noalloc(const smoe_model* model, const smoe_grid* grid, float* image,
                                float* denom, int32_t* status_out, void* stream) {
  clear_stale_error();
  Segs S;
  if (!single_segs(model, grid, &S) || !image) return SMOE_ERR_INVALID;
  const long long cap = static_capacity(model->K, model->C, model->order, S.T);
  if (cap < 0) return SMOE_ERR_TOO_LARGE;
  void* ws = nullptr;
  hipError_t e = static_scratch(&ws);
  if (e != hipSuccess) return hip_status(e);
  smoe_bins b;
  if (layout_into(&b, ws, kStaticScratchBytes, model->K, model->C, model->order, S.T, (int32_t)cap,
                  false) != SMOE_OK)
    return SMOE_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  e = launch_bin(model->C, model->order, model->params, S, b, s);
  if (e == hipSuccess) e = launch_render(model->C, model->order, S, b, image, denom, nullptr, s);
  if (e == hipSuccess && status_out) e = launch_copy_status(b, status_out, s);
  return hip_status(e);
}

smoe_status smoe_materialize(int32_t K, int32_t C, int32_t order, const float* raw, float* model,
                             void* stream) {
  clear_stale_error();
  if (!valid_shape(K, C, order) || (K > 0 && (!raw || !model))) return SMOE_ERR_INVALID;
  return hip_status(launch_materialize(K, C, order, raw, model, static_cast<hipStream_t>(stream)));
}

smoe_status smoe_fit_step(smoe_fit_state* st, const float* target, float* loss_out,
                          void* stream) {
  return fit_step(st, target, loss_out, nullptr, stream);
}

smoe_status smoe_fit_step_timed(smoe_fit_state* st, const float* target, float* loss_out,
                                void* const* stage_events, void* stream) {
  if (!stage_events) return SMOE_ERR_INVALID;
  return fit_step(st, target, loss_out, stage_events, stream);
}

smoe_status smoe_fit_segment_losses(const smoe_fit_state* st, float* out, void* stream) {
  clear_stale_error();
  Segs S;
  if (!st || !out || !st->bins.tile_loss || !fit_segs(st, &S)) return SMOE_ERR_INVALID;
  return hip_status(launch_segment_losses(S, st->bins, out, static_cast<hipStream_t>(stream)));
}

smoe_status smoe_issue_probe(int32_t kind, int32_t iters, int32_t workgroups, float* out,
                             void* stream) {
  clear_stale_error();
  if (kind < 0 || kind > 2 || iters < 1 || workgroups < 1 || workgroups > (1 << 20) || !out)
    return SMOE_ERR_INVALID;
  return hip_status(launch_issue_probe(kind, iters, workgroups, out,
                                       static_cast<hipStream_t>(stream)));
}

smoe_status smoe_fuse_windows(const float* window_images, int32_t C, int32_t width,
                              int32_t height, int32_t window, int32_t displacement,
                              float* image, void* stream) {
  clear_stale_error();
  if ((C != 1 && C != 3) || width < 1 || height < 1 || width > 65536 || height > 65536 ||
      window < 1 || window > 1024 || displacement < 1 || window % displacement != 0 ||
      !window_images || !image)
    return SMOE_ERR_INVALID;
  return hip_status(launch_fuse_windows(window_images, C, width, height, window, displacement,
                                        image, static_cast<hipStream_t>(stream)));
}

smoe_status smoe_pair_stats(const smoe_model* model, const smoe_grid* grid,
                            const smoe_bins* bins, uint64_t* out2, void* stream) {
  clear_stale_error();
  Segs S;
  if (!single_segs(model, grid, &S) || !bins_match(bins, model->K, model->C, model->order) ||
      !out2)
    return SMOE_ERR_INVALID;
  if (S.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  return hip_status(launch_pair_stats(S, *bins, out2, static_cast<hipStream_t>(stream)));
}

smoe_status smoe_read_status(const smoe_bins* bins, int32_t* out4, void* stream) {
  if (!bins || !bins->status) return SMOE_ERR_INVALID;
  int32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return SMOE_ERR_HIP;
  if (hipMemcpy(h, bins->status, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return SMOE_ERR_HIP;
  // word 3: the last binning's non-finite flag; word 7: the fit's (sticky) one
  h[3] = (h[3] || h[7]) ? 1 : 0;
  if (out4) std::memcpy(out4, h, 4 * sizeof(int32_t));
  return h[1] ? SMOE_ERR_CAPACITY : (h[3] ? SMOE_ERR_NONFINITE : SMOE_OK);
}

}  // extern "C"
