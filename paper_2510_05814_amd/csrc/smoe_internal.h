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

// Render record of one kernel, written by the binning pass and staged in LDS by the render
// and backward passes.  Everything a (pixel, kernel) evaluation needs, precomputed once:
//   [0] mu_x  [1] mu_y  [2] i11 = 1/l11  [3] l21  [4] i22 = 1/l22  [5] rho*log2(e)
//   [6] l21*i22  [7 ..] a[C], wx[C], wy[C]
// padded to a multiple of 4 floats so that it moves as float4.
__host__ __device__ constexpr int record_stride(int C, int order) {
  return (7 + expert_floats(C, order) + 3) & ~3;
}
constexpr int kRecExpert = 7;

// Raster description derived from smoe_grid on the host.
struct GridArgs {
  int W, H;        // output pixels
  int scale;       // integer upscale
  int ox, oy;      // origin in output pixels
  float r;         // truncation radius
  float r2;        // r*r, binary32
  float inv_s;     // 1/scale, binary32
  int ntx, nty, T; // blocks
};

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

// Position of kernel j in a block's ascending kernel list vals[lo, hi); -1 if absent.
__device__ __forceinline__ int find_in_list(const uint32_t* __restrict__ vals, int lo, int hi,
                                            uint32_t j) {
  int a = lo, b = hi;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (vals[mid] < j) a = mid + 1;
    else b = mid;
  }
  return (a < hi && vals[a] == j) ? a : -1;
}

// Gradient of parameter i of kernel j: the sum of its per-block partials over the kernel's
// block rectangle in row-major order (a fixed order, so the result is reproducible).  Used
// with 16 lanes per kernel, lane i reading element i of each partial row, so a group's
// reads of one row are contiguous.
template <int NP>
__device__ __forceinline__ float gather_param(int j, int i, int ntx, const int4* __restrict__ rects,
                                              const int2* __restrict__ ranges,
                                              const uint32_t* __restrict__ vals,
                                              const float* __restrict__ pair_grads) {
  float acc = 0.0f;
  const int4 rc = rects[j];
  for (int ty = rc.y; ty <= rc.w; ++ty)
    for (int tx = rc.x; tx <= rc.z; ++tx) {
      const int2 rg = ranges[ty * ntx + tx];
      if (rg.y <= rg.x) continue;
      const int p = find_in_list(vals, rg.x, rg.y, (uint32_t)j);
      if (p >= 0 && i < NP) acc += pair_grads[(size_t)p * NP + i];
    }
  return acc;
}

hipError_t launch_bin(const smoe_model& m, const GridArgs& g, const smoe_bins& b, hipStream_t s);
// Fit-step pieces: block counters, boxes and records of the current model (fill,
// preprocess); the scan of the counters into ranges; the scatter into buckets; the fused
// per-block sort + render + backward; Adam fused with the next step's boxes, records and
// counters.
hipError_t launch_count(const smoe_model& m, const GridArgs& g, const smoe_bins& b,
                        hipStream_t s);
// fit_step (the fit step only): the step counter to snapshot for the step's Adam kernel.
hipError_t launch_scan(const GridArgs& g, const smoe_bins& b, hipStream_t s,
                       const int32_t* fit_step = nullptr);
hipError_t launch_scatter(const smoe_model& m, const GridArgs& g, const smoe_bins& b,
                          hipStream_t s);
hipError_t launch_fit_tile(const smoe_fit_state& st, const GridArgs& g, const float* target,
                           hipStream_t s);
hipError_t launch_adam_fit(const smoe_fit_state& st, const GridArgs& g, float* loss_out,
                           hipStream_t s);
hipError_t launch_render(const smoe_model& m, const GridArgs& g, const smoe_bins& b, float* image,
                         float* denom, const float* target, hipStream_t s);
hipError_t launch_pair_stats(const smoe_model& m, const GridArgs& g, const smoe_bins& b,
                             uint64_t* out2, hipStream_t s);
hipError_t launch_loss_reduce(const smoe_bins& b, int T, float inv_n, float* loss_out,
                              hipStream_t s);
hipError_t launch_backward(const smoe_model& m, const GridArgs& g, const smoe_bins& b,
                           const float* image, const float* denom, const float* grad_image,
                           const float* target, hipStream_t s);
hipError_t launch_gather(const smoe_model& m, const GridArgs& g, const smoe_bins& b, float* grads,
                         hipStream_t s);
hipError_t launch_materialize(int K, int C, int order, const float* raw, float* model,
                              hipStream_t s);

}  // namespace smoe
