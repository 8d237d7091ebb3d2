// Backward (adjoint) of the rasterized SMoE render on gfx950: the standalone call.
//
// Nothing per (pixel, kernel) is stored by the forward: for every pixel the backward
// recomputes each participating kernel's gate term pi K from the record and divides by the
// saved denominator D, then forms the adjoints of all 6 + 3C raw parameters (formulas in
// tile_math.h).  Pixels outside the ellipse or the kernel's blocks contribute nothing
// (Sec. IV-B).
//
// Work split: one wave per 16x16 block.  Per kernel the wave's per-lane sums are reduced over
// the block's 256 pixels by a transposed butterfly (cross-half swaps, then DPP) into one
// per-(block, kernel) partial row.  A second pass sums each kernel's partial rows over its
// blocks in row-major block order.  Every order is fixed: gradients are bitwise
// reproducible and no atomics are used.
#include "tile_math.h"

namespace smoe {
namespace {

struct BackwardArgs {
  GridArgs g;
  const float* __restrict__ records;
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  const float* __restrict__ image;
  const float* __restrict__ denom;
  const float* __restrict__ grad_image;  // upstream dL/dy, or null
  const float* __restrict__ target;      // MSE target, or null
  float inv_n2;                          // 2 / (W H C) for the MSE
  float* __restrict__ pair_grads;
};

template <int C, int ORDER>
__global__ __launch_bounds__(kWave) void k_backward(BackwardArgs a) {
  __shared__ float4 srec[kChunk * record_stride(C, ORDER) / 4];
  const int tile = xcd_block(blockIdx.x, a.g.T);
  const PixelCoords px = lane_pixels(a.g, tile);
  PixelSeed<C> sd;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int v = px.v0 + 4 * i;
    sd.valid[i] = false;
    sd.invD[i] = 0.0f;
    sd.gy[i] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) sd.g[i][c] = 0.0f;
    if (px.u < a.g.W && v < a.g.H) {
      const size_t p = (size_t)v * a.g.W + px.u;
      const float D = a.denom[p];
      if (D > 0.0f) {
        sd.valid[i] = true;
        sd.invD[i] = 1.0f / D;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const float yc = a.image[p * C + c];
          sd.g[i][c] = a.target ? (yc - a.target[p * C + c]) * a.inv_n2 : a.grad_image[p * C + c];
          sd.gy[i] = __builtin_fmaf(sd.g[i][c], yc, sd.gy[i]);
        }
      }
    }
  }
  backward_accumulate<C, ORDER>(px, a.g.r2, a.records, a.vals, a.ranges[tile], srec, false, sd,
                                a.pair_grads);
}

struct GatherArgs {
  int K;
  int ntx;
  const int4* __restrict__ tile_rects;
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  const float* __restrict__ pair_grads;
  const int32_t* __restrict__ status;
  float* __restrict__ grads;
};

// 16 lanes per kernel: lane i of the group reduces parameter i.
template <int NP>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = gid >> 4, i = gid & 15;
  if (j >= a.K) return;
  const float g = a.status[1] != 0
                      ? 0.0f
                      : gather_param<NP>(j, i, a.ntx, a.tile_rects, a.ranges, a.vals, a.pair_grads);
  if (i < NP) a.grads[(size_t)j * NP + i] = g;
}

}  // namespace

hipError_t launch_backward(const smoe_model& m, const GridArgs& g, const smoe_bins& b,
                           const float* image, const float* denom, const float* grad_image,
                           const float* target, hipStream_t s) {
  BackwardArgs a{g,
                 b.records,
                 reinterpret_cast<const int2*>(b.ranges),
                 b.vals,
                 image,
                 denom,
                 grad_image,
                 target,
                 2.0f / ((float)g.W * (float)g.H * (float)m.C),
                 b.pair_grads};
  if (m.C == 1 && m.order == 0) k_backward<1, 0><<<g.T, kWave, 0, s>>>(a);
  else if (m.C == 1 && m.order == 1) k_backward<1, 1><<<g.T, kWave, 0, s>>>(a);
  else if (m.C == 3 && m.order == 0) k_backward<3, 0><<<g.T, kWave, 0, s>>>(a);
  else k_backward<3, 1><<<g.T, kWave, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_gather(const smoe_model& m, const GridArgs& g, const smoe_bins& b, float* grads,
                         hipStream_t s) {
  if (m.K == 0) return hipSuccess;
  GatherArgs a{m.K,
               g.ntx,
               reinterpret_cast<const int4*>(b.tile_rects),
               reinterpret_cast<const int2*>(b.ranges),
               b.vals,
               b.pair_grads,
               b.status,
               grads};
  const int blocks = (int)(((long long)m.K * 16 + 255) / 256);
  const int NP = num_params(m.C, m.order);
  if (NP == 7) k_gather<7><<<blocks, 256, 0, s>>>(a);
  else if (NP == 9) k_gather<9><<<blocks, 256, 0, s>>>(a);  // (C, order) = (1, 1) or (3, 0)
  else k_gather<15><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace smoe
