// The C ABI of include/smoe.h: host-side validation, workspace layout and the launch
// sequences of each call.  No device memory is allocated here.
#include <cmath>
#include <cstring>

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

bool make_grid(const smoe_grid* g, GridArgs* out) {
  if (!g) return false;
  if (g->width < 1 || g->height < 1 || g->width > 65536 || g->height > 65536) return false;
  if (g->scale < 1 || g->scale > 64) return false;
  if (std::abs(g->origin_x) > (1 << 22) || std::abs(g->origin_y) > (1 << 22)) return false;
  if (!(g->radius > 0.0f) || !std::isfinite(g->radius)) return false;
  GridArgs a;
  a.W = g->width;
  a.H = g->height;
  a.scale = g->scale;
  a.ox = g->origin_x;
  a.oy = g->origin_y;
  a.r = g->radius;
  a.r2 = g->radius * g->radius;
  a.inv_s = 1.0f / (float)g->scale;
  a.ntx = (g->width + kTile - 1) / kTile;
  a.nty = (g->height + kTile - 1) / kTile;
  a.T = a.ntx * a.nty;
  *out = a;
  return true;
}

bool bins_match(const smoe_bins* b, const smoe_model* m) {
  return b && b->K == m->K && b->C == m->C && b->order == m->order && b->status &&
         b->ranges && b->vals && b->records;
}

struct Layout {
  size_t tile_rects, counts, records, tile_counts, ranges, keys, vals, vals_alt, pair_grads,
      tile_loss, status, total;
};

Layout layout_of(int32_t K, int32_t C, int32_t order, int32_t max_tiles, int32_t capacity) {
  const size_t rs = (size_t)record_stride(C, order);
  const size_t np = (size_t)num_params(C, order);
  Layout L;
  size_t o = 0;
  L.tile_rects = o; o = align_up(o + (size_t)K * 4 * sizeof(int32_t));
  L.counts = o;     o = align_up(o + (size_t)K * sizeof(int32_t));
  L.records = o;    o = align_up(o + (size_t)K * rs * sizeof(float));
  L.tile_counts = o; o = align_up(o + (size_t)max_tiles * sizeof(int32_t));
  L.ranges = o;     o = align_up(o + (size_t)max_tiles * 2 * sizeof(int32_t));
  L.keys = o;       o = align_up(o + (size_t)capacity * sizeof(uint32_t));
  L.vals = o;       o = align_up(o + (size_t)capacity * sizeof(uint32_t));
  L.vals_alt = o;   o = align_up(o + (size_t)capacity * sizeof(uint32_t));
  L.pair_grads = o; o = align_up(o + (size_t)capacity * np * sizeof(float));
  L.tile_loss = o;  o = align_up(o + (size_t)max_tiles * sizeof(float));
  L.status = o;     o = align_up(o + 8 * sizeof(int32_t));
  L.total = o;
  return L;
}

inline smoe_status hip_status(hipError_t e) { return e == hipSuccess ? SMOE_OK : SMOE_ERR_HIP; }

}  // namespace

extern "C" {

int32_t smoe_version(void) { return 100; }

size_t smoe_bins_workspace_bytes(int32_t K, int32_t C, int32_t order, int32_t max_tiles,
                                 int32_t capacity) {
  if (!valid_shape(K, C, order) || max_tiles < 1 || capacity < 0) return 0;
  return layout_of(K, C, order, max_tiles, capacity).total;
}

smoe_status smoe_bins_layout(smoe_bins* out, void* workspace, size_t bytes, int32_t K, int32_t C,
                             int32_t order, int32_t max_tiles, int32_t capacity) {
  if (!out || !workspace || !valid_shape(K, C, order) || max_tiles < 1 || capacity < 0)
    return SMOE_ERR_INVALID;
  if (((uintptr_t)workspace & (kAlign - 1)) != 0) return SMOE_ERR_INVALID;
  const Layout L = layout_of(K, C, order, max_tiles, capacity);
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
  b.counts = reinterpret_cast<int32_t*>(base + L.counts);
  b.records = reinterpret_cast<float*>(base + L.records);
  b.record_stride = record_stride(C, order);
  b.tile_counts = reinterpret_cast<int32_t*>(base + L.tile_counts);
  b.ranges = reinterpret_cast<int32_t*>(base + L.ranges);
  b.keys = reinterpret_cast<uint32_t*>(base + L.keys);
  b.vals = reinterpret_cast<uint32_t*>(base + L.vals);
  b.vals_alt = reinterpret_cast<uint32_t*>(base + L.vals_alt);
  b.pair_grads = reinterpret_cast<float*>(base + L.pair_grads);
  b.tile_loss = reinterpret_cast<float*>(base + L.tile_loss);
  b.status = reinterpret_cast<int32_t*>(base + L.status);
  *out = b;
  return SMOE_OK;
}

smoe_status smoe_bin(const smoe_model* model, const smoe_grid* grid, smoe_bins* bins,
                     void* stream) {
  GridArgs g;
  if (!valid_model(model) || !make_grid(grid, &g) || !bins_match(bins, model))
    return SMOE_ERR_INVALID;
  if (g.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  return hip_status(launch_bin(*model, g, *bins, static_cast<hipStream_t>(stream)));
}

smoe_status smoe_render(const smoe_model* model, const smoe_grid* grid, const smoe_bins* bins,
                        float* image, float* denom, const float* target, float* loss_out,
                        void* stream) {
  GridArgs g;
  if (!valid_model(model) || !make_grid(grid, &g) || !bins_match(bins, model) || !image)
    return SMOE_ERR_INVALID;
  if (g.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  const bool loss = target && loss_out;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_render(*model, g, *bins, image, denom, loss ? target : nullptr, s);
  if (e == hipSuccess && loss) {
    const float inv_n = (float)(1.0 / ((double)g.W * g.H * model->C));
    e = launch_loss_reduce(*bins, g.T, inv_n, loss_out, s);
  }
  return hip_status(e);
}

smoe_status smoe_render_backward(const smoe_model* model, const smoe_grid* grid,
                                 const smoe_bins* bins, const float* image, const float* denom,
                                 const float* grad_image, const float* target, float* grads,
                                 void* stream) {
  GridArgs g;
  if (!valid_model(model) || !make_grid(grid, &g) || !bins_match(bins, model) || !image ||
      !denom || !grads || (grad_image == nullptr) == (target == nullptr) || !bins->pair_grads)
    return SMOE_ERR_INVALID;
  if (g.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_backward(*model, g, *bins, image, denom, grad_image, target, s);
  if (e == hipSuccess) e = launch_gather(*model, g, *bins, grads, s);
  return hip_status(e);
}

smoe_status smoe_materialize(int32_t K, int32_t C, int32_t order, const float* raw, float* model,
                             void* stream) {
  if (!valid_shape(K, C, order) || (K > 0 && (!raw || !model))) return SMOE_ERR_INVALID;
  return hip_status(launch_materialize(K, C, order, raw, model, static_cast<hipStream_t>(stream)));
}

namespace {

smoe_status fit_step(smoe_fit_state* st, const float* target, float* loss_out,
                     void* const* ev, void* stream) {
  if (!st || !target) return SMOE_ERR_INVALID;
  const smoe_model m{st->K, st->C, st->order, st->model};
  GridArgs g;
  if (!valid_model(&m) || !make_grid(&st->grid, &g) || !bins_match(&st->bins, &m))
    return SMOE_ERR_INVALID;
  if (st->grid.scale != 1 || st->grid.origin_x != 0 || st->grid.origin_y != 0)
    return SMOE_ERR_INVALID;
  if (!st->raw || !st->adam_m || !st->adam_v || !st->image || !st->denom || !st->step ||
      !st->scalars || !st->bins.pair_grads || !st->bins.tile_loss)
    return SMOE_ERR_INVALID;
  if (st->max_steps < 0) return SMOE_ERR_INVALID;
  if (g.T > st->bins.max_tiles) return SMOE_ERR_TOO_LARGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto mark = [&](int i) -> hipError_t {
    return (ev && ev[i]) ? hipEventRecord(static_cast<hipEvent_t>(ev[i]), s) : hipSuccess;
  };
  hipError_t e = mark(0);
  if (e == hipSuccess && !st->prepared) e = launch_count(m, g, st->bins, s);
  if (e == hipSuccess) e = launch_scan(g, st->bins, s, st->step);
  if (e == hipSuccess) e = launch_scatter(m, g, st->bins, s);
  if (e == hipSuccess) e = mark(1);
  if (e == hipSuccess) e = launch_fit_tile(*st, g, target, s);
  if (e == hipSuccess) e = mark(2);
  if (e == hipSuccess) e = launch_adam_fit(*st, g, loss_out, s);
  if (e == hipSuccess) e = mark(3);
  if (e == hipSuccess) st->prepared = 1;
  return hip_status(e);
}

}  // namespace

smoe_status smoe_fit_step(smoe_fit_state* st, const float* target, float* loss_out,
                          void* stream) {
  return fit_step(st, target, loss_out, nullptr, stream);
}

smoe_status smoe_fit_step_timed(smoe_fit_state* st, const float* target, float* loss_out,
                                void* const* stage_events, void* stream) {
  if (!stage_events) return SMOE_ERR_INVALID;
  return fit_step(st, target, loss_out, stage_events, stream);
}

smoe_status smoe_pair_stats(const smoe_model* model, const smoe_grid* grid,
                            const smoe_bins* bins, uint64_t* out2, void* stream) {
  GridArgs g;
  if (!valid_model(model) || !make_grid(grid, &g) || !bins_match(bins, model) || !out2)
    return SMOE_ERR_INVALID;
  if (g.T > bins->max_tiles) return SMOE_ERR_TOO_LARGE;
  return hip_status(launch_pair_stats(*model, g, *bins, out2, static_cast<hipStream_t>(stream)));
}

smoe_status smoe_read_status(const smoe_bins* bins, int32_t* out4, void* stream) {
  if (!bins || !bins->status) return SMOE_ERR_INVALID;
  int32_t h[4] = {0, 0, 0, 0};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return SMOE_ERR_HIP;
  if (hipMemcpy(h, bins->status, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return SMOE_ERR_HIP;
  if (out4) std::memcpy(out4, h, sizeof(h));
  return h[1] ? SMOE_ERR_CAPACITY : SMOE_OK;
}

}  // extern "C"
