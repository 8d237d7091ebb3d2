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
  Segs S;
  int C;
  const float* __restrict__ records;
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  const float* __restrict__ image;
  const float* __restrict__ denom;
  const float* __restrict__ grad_image;  // upstream dL/dy, or null
  const float* __restrict__ target;      // MSE target, or null
  float* __restrict__ pair_grads;
};

template <int C, int ORDER, bool RBF>
__global__ __launch_bounds__(kWave) void k_backward(BackwardArgs a) {
  __shared__ float4 srec[kChunk * record_stride(C, ORDER) / 4];
  const int tile = xcd_block(blockIdx.x, a.S.T);
  const SegGrid sg = seg_of_tile(a.S, tile);
  const PixelCoords px = lane_pixels(sg, tile - sg.tile_offset);
  // MSE of this raster: dL/dy = 2 (y - t) / (W H C)
  const float inv_n2 = 2.0f / ((float)sg.W * (float)sg.H * (float)C);
  PixelSeed<C> sd;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int v = px.v0 + 4 * i;
    sd.valid[i] = false;
    sd.invD[i] = 0.0f;
    sd.gy[i] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) sd.g[i][c] = 0.0f;
    if (in_raster(px.u, v, sg)) {
      const size_t p = (size_t)sg.pixel_offset + (size_t)v * sg.W + px.u;
      const float D = a.denom[p];
      if (D > 0.0f) {
        sd.valid[i] = true;
        sd.invD[i] = RBF ? 1.0f : __builtin_amdgcn_rcpf(D);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const float yc = a.image[p * C + c];
          sd.g[i][c] = a.target ? (yc - a.target[p * C + c]) * inv_n2 : a.grad_image[p * C + c];
          if (!RBF) sd.gy[i] = __builtin_fmaf(sd.g[i][c], yc, sd.gy[i]);
        }
      }
    }
  }
  backward_accumulate<C, ORDER>(px, a.S.r2, a.records, a.vals, 0, false, a.ranges[tile], srec,
                                false, 0ull, sd, a.pair_grads);
}

struct GatherArgs {
  Segs S;
  const float* __restrict__ records;
  const int4* __restrict__ tile_rects;
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  const float* __restrict__ pair_grads;
  const int32_t* __restrict__ status;
  float* __restrict__ grads;
};

// 16 lanes per kernel (one 16-lane row of the wave); lane i ends with parameter i.
template <int C, int ORDER>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
  constexpr int NP = num_params(C, ORDER);
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = gid >> 4, i = gid & 15;
  constexpr int RS = record_stride(C, ORDER);
  const bool live = j < a.S.K;
  const float rec = live && i < RS ? a.records[(size_t)j * RS + i] : 0.0f;
  // every lane takes part in the gather's row reduction and the finishing shuffles
  const float s = gather_param<NP>(j, live && a.status[1] == 0, seg_of_kernel(a.S, live ? j : 0),
                                   a.tile_rects, a.ranges, a.vals, a.pair_grads);
  const float g = finish_gradient<C, ORDER, kRecExpert>(s, live, rec);
  if (live && i < NP) a.grads[(size_t)j * NP + i] = g;
}

}  // namespace

hipError_t launch_backward(int C, int order, const Segs& S, const smoe_bins& b,
                           const float* image, const float* denom, const float* grad_image,
                           const float* target, hipStream_t s) {
  BackwardArgs a{S,
                 C,
                 b.records,
                 reinterpret_cast<const int2*>(b.ranges),
                 b.vals,
                 image,
                 denom,
                 grad_image,
                 target,
                 b.pair_grads};
  with_shape(C, order, S, [&](auto sh) {
    using T = decltype(sh);
    k_backward<T::C, T::ORDER, T::RBF><<<S.T, kWave, 0, s>>>(a);
  });
  return hipGetLastError();
}

hipError_t launch_gather(int C, int order, const Segs& S, const smoe_bins& b, float* grads,
                         hipStream_t s) {
  if (S.K == 0) return hipSuccess;
  GatherArgs a{S,
               b.records,
               reinterpret_cast<const int4*>(b.tile_rects),
               reinterpret_cast<const int2*>(b.ranges),
               b.vals,
               b.pair_grads,
               b.status,
               grads};
  const int blocks = (int)(((long long)S.K * 16 + 255) / 256);
  if (C == 1 && order == 0) k_gather<1, 0><<<blocks, 256, 0, s>>>(a);
  else if (C == 1 && order == 1) k_gather<1, 1><<<blocks, 256, 0, s>>>(a);
  else if (C == 3 && order == 0) k_gather<3, 0><<<blocks, 256, 0, s>>>(a);
  else k_gather<3, 1><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace smoe
