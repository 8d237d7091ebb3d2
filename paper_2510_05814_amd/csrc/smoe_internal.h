// Internal declarations of the gfx950 SMoE library: device helpers shared by the kernels
// and the launchers that the C ABI (capi.hip) calls.  Not a public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smoe.h"

namespace smoe {

constexpr int kTile = 16;
constexpr int kTilePixels = kTile * kTile;
constexpr float kLog2e = 1.44269504088896340736f;

// Expert coefficients per kernel: a[C] (+ wx[C], wy[C] for linear experts).
__host__ __device__ constexpr int expert_floats(int C, int order) { return C * (1 + 2 * order); }
__host__ __device__ constexpr int num_params(int C, int order) { return 6 + expert_floats(C, order); }
// Floats per per-(block, kernel) gradient partial row: NP rounded up to a multiple of 4, so
// that every row starts on 16 bytes and moves as float4.
__host__ __device__ constexpr int partial_stride(int np) { return (np + 3) & ~3; }

// Render record of one kernel, written by the binning pass and staged in LDS by the render
// and backward passes.  Everything a (pixel, kernel) evaluation needs, precomputed once:
//   [0] mu_x  [1] mu_y  [2] i11 = 1/l11  [3] l21  [4] i22 = 1/l22  [5] rho*log2(e)
//   [6] l21*i22  [7 ..] a[C], wx[C], wy[C]
// padded to a multiple of 4 floats so that it moves as float4.
__host__ __device__ constexpr int record_stride(int C, int order) {
  return (7 + expert_floats(C, order) + 3) & ~3;
}
constexpr int kRecExpert = 7;

// The rasters of one call.  A batched call (several images of a batched fit, or several
// render requests) numbers the blocks of all its rasters consecutively (segment s owns
// blocks [tile_offset, tile_offset + T_s)) and its kernel rows likewise; each kernel and
// each block then finds its segment by a binary search on those offsets.  A single-raster
// call has no table (tab == null) and uses `one`.
struct Segs {
  const smoe_segment* __restrict__ tab;  // device table of n segments, or null
  int n;
  smoe_segment one;                      // the single raster when tab is null
  float r, r2;                           // truncation radius and r*r (binary32)
  float r2_render;                       // the render's bound on q: r2 (ellipse in the
                                         // render), or 0 (no bound on q)
  // The render's bound applied without a compare.  Ellipse in the render: with
  // cut_scale = 2^k such that r2_render * 2^k lies in [2^60, 2^61) and
  // cut_offset = -r2_render * 2^k (both exact), u = fma(q, cut_scale, cut_offset) is <= 0 for
  // q <= r2_render and >= 2^37 beyond it, so max(q, u) is q inside the bound and pushes the
  // exponent of a term beyond it to about -2^36, whose exp2 is exactly zero.  Block lists
  // deciding the render: cut_scale = 2^60, cut_offset = 125 * 2^60, and for the term's
  // exponent a, min(a, fma(a, cut_scale, cut_offset)) is a when a >= -125 (the term is a
  // normal binary32 number) and below -2^43 otherwise.
  float cut_scale, cut_offset;
  int box;                               // SMOE_BOX_SQUARE or SMOE_BOX_TIGHT
  int mode;                              // SMOE_MODE_SMOE or SMOE_MODE_RBF
  int trunc;                             // SMOE_TRUNC_RENDER or SMOE_TRUNC_GRADIENT
  int T;                                 // blocks of all segments
  int K;                                 // kernel rows of all segments
};

// Blocks of a raster: the 16x16 blocks of the output grid of its scale, aligned to
// multiples of 16 in the output coordinate o + u (so that at scale s a native block, 16 s
// output pixels, is a whole number of blocks); a window's first and last blocks may be
// partial on either side.  first_block(o) = floor(o / 16) is the grid block of the raster's
// first pixel; blocks_across(n, o) the blocks its n pixels touch.
__host__ __device__ constexpr int first_block(int o) { return o >= 0 ? o / 16 : -((15 - o) / 16); }
__host__ __device__ constexpr int blocks_across(int n, int o) {
  return first_block(o + n - 1) - first_block(o) + 1;
}

// One segment's raster, as the kernels use it.
struct SegGrid {
  int W, H, scale, ox, oy, ntx;
  int bx0, by0;                // grid block of the raster's first pixel, per axis
  float inv_s;                 // 1/scale, binary32
  int tile_offset, kernel_offset, param_offset, K;
  long long pixel_offset;
  float sharpen;               // bandwidth divisor, 1 = none
};

__host__ __device__ inline SegGrid seg_grid_of(const smoe_segment& s) {
  SegGrid g;
  g.W = s.width;
  g.H = s.height;
  g.scale = s.scale;
  g.ox = s.origin_x;
  g.oy = s.origin_y;
  g.ntx = blocks_across(s.width, s.origin_x);
  g.bx0 = first_block(s.origin_x);
  g.by0 = first_block(s.origin_y);
  g.inv_s = 1.0f / (float)s.scale;
  g.tile_offset = s.tile_offset;
  g.kernel_offset = s.kernel_offset;
  g.param_offset = s.param_offset;
  g.K = s.num_kernels;
  g.pixel_offset = s.pixel_offset;
  g.sharpen = s.sharpen > 0.0f ? s.sharpen : 1.0f;
  return g;
}

// Segment of global block t: the last segment whose tile_offset <= t.
__device__ __forceinline__ SegGrid seg_of_tile(const Segs& S, int t) {
  if (!S.tab) return seg_grid_of(S.one);
  int lo = 0, hi = S.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (S.tab[mid].tile_offset <= t) lo = mid;
    else hi = mid - 1;
  }
  return seg_grid_of(S.tab[lo]);
}

// Segment of global kernel row j: the last segment whose kernel_offset <= j (segments
// without kernels share their offset with the next one and are skipped by "last").
__device__ __forceinline__ SegGrid seg_of_kernel(const Segs& S, int j) {
  if (!S.tab) return seg_grid_of(S.one);
  int lo = 0, hi = S.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (S.tab[mid].kernel_offset <= j) lo = mid;
    else hi = mid - 1;
  }
  return seg_grid_of(S.tab[lo]);
}

// Output pixel index -> native sampling coordinate, the exact binary32 sequence of the
// ABI contract: ((o + u) + 0.5) * inv_s.
__device__ __forceinline__ float sample_coord(int u, int o, float inv_s) {
  return ((float)(o + u) + 0.5f) * inv_s;
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8).
// Remap so that each XCD walks one contiguous band of blocks: neighbouring blocks share
// most of their kernels, so their records then stay in that XCD's L2.  A bijection on
// [0, T): the first 8*floor(T/8) ids are permuted, the tail maps to itself.
__device__ __forceinline__ int xcd_block(int b, int T) {
  const int full = T & ~7;
  if (b >= full) return b;
  const int per = T >> 3;
  return (b & 7) * per + (b >> 3);
}

// Position of kernel j in a block's ascending kernel list vals[lo, hi); -1 if absent.  An
// entry holds the kernel id shifted left by `shift` (the fit step's buckets keep the row of
// the entry's gradient partial in the low bits).
__device__ __forceinline__ int find_in_list(const uint32_t* __restrict__ vals, int lo, int hi,
                                            uint32_t j, int shift = 0) {
  int a = lo, b = hi;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if ((vals[mid] >> shift) < j) a = mid + 1;
    else b = mid;
  }
  return (a < hi && (vals[a] >> shift) == j) ? a : -1;
}

// The fit step stores the gradient partial row of kernel j in its block q (row-major in its
// block rectangle) at row kSlots j + q of the pair storage when q < kSlots -- each kernel's
// first blocks are kernel-major, so its gradient gather reads them contiguously -- and at row
// kSlots K + the entry's bucket slot for the kernel's further blocks.
constexpr int kSlots = 16;

// Launchers.  `params` rows are addressed through each segment's param_offset; every
// per-kernel workspace array through kernel_offset; images through pixel_offset.
hipError_t launch_bin(int C, int order, const float* params, const Segs& S, const smoe_bins& b,
                      hipStream_t s);
hipError_t launch_render(int C, int order, const Segs& S, const smoe_bins& b, float* image,
                         float* denom, const float* target, hipStream_t s);
hipError_t launch_pair_stats(const Segs& S, const smoe_bins& b, uint64_t* out2, hipStream_t s);
hipError_t launch_loss_reduce(const smoe_bins& b, int T, float inv_n, float* loss_out,
                              hipStream_t s);
hipError_t launch_backward(int C, int order, const Segs& S, const smoe_bins& b,
                           const float* image, const float* denom, const float* grad_image,
                           const float* target, hipStream_t s);
hipError_t launch_gather(int C, int order, const Segs& S, const smoe_bins& b, float* grads,
                         hipStream_t s);
hipError_t launch_materialize(int K, int C, int order, const float* raw, float* model,
                              hipStream_t s);
// Binning pieces: block counters, boxes and records of the current model (fill,
// preprocess); the scan of the counters into ranges; the scatter into the lists.
hipError_t launch_count(int C, int order, const float* params, const Segs& S,
                        const smoe_bins& b, hipStream_t s);
hipError_t launch_scan(const Segs& S, const smoe_bins& b, hipStream_t s);
hipError_t launch_scatter(const Segs& S, const smoe_bins& b, hipStream_t s);
// Copies the first four status words (P needed, overflow, longest list, spare) to out4.
hipError_t launch_copy_status(const smoe_bins& b, int32_t* out4, hipStream_t s);
// Fit step: boxes and records of the current model with zeroed bucket cursors and status
// words (the first step); then every step the scatter into fixed-width buckets (over each
// kernel's box, computed from its model row), the fused per-block sort + render + backward,
// and Adam fused with the re-materialization and the next step's render records.
hipError_t launch_prepare_fit(int C, int order, const float* params, const Segs& S,
                              const smoe_bins& b, hipStream_t s);
// The fit step's bucket entries: kernel id << shift | the row of the entry's gradient
// partial (kSlots + width <= 2^shift).
hipError_t launch_scatter_fixed(const Segs& S, const smoe_bins& b, const float* model, int np,
                                int width, int shift, const int32_t* step,
                                const smoe_adam_config& adam, float* scalars, hipStream_t s);
hipError_t launch_fit_tile(const smoe_fit_state& st, const Segs& S, int width, int shift,
                           const float* target, hipStream_t s);
hipError_t launch_adam_fit(const smoe_fit_state& st, const Segs& S, int shift, float* loss_out,
                           hipStream_t s);
hipError_t launch_segment_losses(const Segs& S, const smoe_bins& b, float* out, hipStream_t s);
hipError_t launch_issue_probe(int kind, int iters, int workgroups, float* out, hipStream_t s);
hipError_t launch_fuse_windows(const float* windows, int C, int width, int height, int window,
                               int d, float* image, hipStream_t s);

}  // namespace smoe
