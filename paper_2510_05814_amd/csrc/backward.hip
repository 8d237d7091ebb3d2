// Backward (adjoint) of the rasterized SMoE render on gfx950.
//
// Nothing per (pixel, kernel) is stored by the forward: for every pixel the backward
// recomputes each participating kernel's gate term e = pi K from the record and divides by
// the saved denominator D, so w = e / D, then forms the adjoints of all 6 + 3C raw
// parameters.  With g_c = dL/dy_c at the pixel:
//   G = sum_c g_c (m_c - y_c),  H = w G                       (dL/drho)
//   dL/da_c = g_c w,  dL/dwx_c = g_c w dx,  dL/dwy_c = g_c w dy
//   bz2 = -H z2,  bz1 = -H z1 - bz2 l21/l22                  (through q = z1^2 + z2^2)
//   dL/dmu_x = -(bz1/l11 + sum_c g_c w wx_c),  dL/dmu_y = -(bz2/l22 + sum_c g_c w wy_c)
//   dL/ds1 = -bz1 z1,  dL/dl21 = -bz2 z1/l22,  dL/ds2 = -bz2 z2
// Pixels outside the ellipse or the kernel's blocks contribute nothing (Sec. IV-B).
//
// Reduction: one workgroup per block, one pixel per lane; per kernel the workgroup sums the
// 6+3C per-lane values (wave butterfly, then the 4 wave partials in a fixed order) into
// one per-(block, kernel) partial row.  A second pass sums each kernel's partial rows over
// its blocks in row-major block order.  Both orders are fixed, so gradients are bitwise
// reproducible and no atomics are used.
#include "smoe_internal.h"

namespace smoe {
namespace {

constexpr int kThreads = kTilePixels;

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

template <int RS>
__device__ __forceinline__ void stage_records(float4* __restrict__ srec,
                                              const float* __restrict__ records,
                                              const uint32_t* __restrict__ vals, int base, int n) {
  constexpr int Q = RS / 4;
  for (int i = threadIdx.x; i < n * Q; i += kThreads) {
    const int k = i / Q, c = i - k * Q;
    const uint32_t j = vals[base + k];
    srec[i] = reinterpret_cast<const float4*>(records + (size_t)j * RS)[c];
  }
}

template <int C, int ORDER>
__global__ __launch_bounds__(kThreads) void k_backward(BackwardArgs a) {
  constexpr int RS = record_stride(C, ORDER);
  constexpr int NP = num_params(C, ORDER);
  __shared__ float4 srec[kThreads * RS / 4];
  __shared__ float sred[kThreads / 64][NP];

  const int tile = xcd_block(blockIdx.x, a.g.T);
  const int tx = tile % a.g.ntx, ty = tile / a.g.ntx;
  const int u = tx * kTile + (threadIdx.x & 15);
  const int v = ty * kTile + (threadIdx.x >> 4);
  const float x = sample_coord(u, a.g.ox, a.g.inv_s);
  const float y = sample_coord(v, a.g.oy, a.g.inv_s);
  const float r2 = a.g.r2;
  const int2 rg = a.ranges[tile];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // Per-pixel adjoint seed.
  bool valid = false;
  float invD = 0.0f, gy = 0.0f;
  float g[C];
#pragma unroll
  for (int c = 0; c < C; ++c) g[c] = 0.0f;
  if (u < a.g.W && v < a.g.H) {
    const size_t p = (size_t)v * a.g.W + u;
    const float D = a.denom[p];
    if (D > 0.0f) {
      valid = true;
      invD = 1.0f / D;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float yc = a.image[p * C + c];
        g[c] = a.target ? (yc - a.target[p * C + c]) * a.inv_n2 : a.grad_image[p * C + c];
        gy = __builtin_fmaf(g[c], yc, gy);
      }
    }
  }

  for (int base = rg.x; base < rg.y; base += kThreads) {
    const int n = min(kThreads, rg.y - base);
    __syncthreads();
    stage_records<RS>(srec, a.records, a.vals, base, n);
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const float* r = reinterpret_cast<const float*>(&srec[k * (RS / 4)]);
      float acc[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) acc[i] = 0.0f;
      const float dx = x - r[0];
      const float dy = y - r[1];
      const float z1 = dx * r[2];
      const float tt = r[3] * z1;
      const float w_ = dy - tt;
      const float z2 = w_ * r[4];
      const float q = z1 * z1 + z2 * z2;
      if (valid && q <= r2) {
        const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(q, -0.5f * kLog2e, r[5]));
        const float w = e * invD;
        float Gs = -gy;
        float ex = 0.0f, ey = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          float m = r[kRecExpert + c];
          if (ORDER == 1) {
            m = __builtin_fmaf(r[kRecExpert + C + c], dx, m);
            m = __builtin_fmaf(r[kRecExpert + 2 * C + c], dy, m);
          }
          Gs = __builtin_fmaf(g[c], m, Gs);
          const float gw = g[c] * w;
          acc[6 + c] = gw;
          if (ORDER == 1) {
            acc[6 + C + c] = gw * dx;
            acc[6 + 2 * C + c] = gw * dy;
            ex = __builtin_fmaf(gw, r[kRecExpert + C + c], ex);
            ey = __builtin_fmaf(gw, r[kRecExpert + 2 * C + c], ey);
          }
        }
        const float Hh = w * Gs;
        const float bz2 = -Hh * z2;
        const float bz1 = __builtin_fmaf(-bz2, r[6], -Hh * z1);
        acc[0] = -__builtin_fmaf(bz1, r[2], ex);
        acc[1] = -__builtin_fmaf(bz2, r[4], ey);
        acc[2] = -bz1 * z1;
        acc[3] = -bz2 * z1 * r[4];
        acc[4] = -bz2 * z2;
        acc[5] = Hh;
      }
      // Workgroup sum of the NP values: wave butterfly, then waves 0..3 in order.
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        float t = acc[i];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
        acc[i] = t;
      }
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i) sred[wave][i] = acc[i];
      }
      __syncthreads();
      if (threadIdx.x < NP) {
        const int i = threadIdx.x;
        a.pair_grads[(size_t)(base + k) * NP + i] = (sred[0][i] + sred[1][i]) + (sred[2][i] + sred[3][i]);
      }
      __syncthreads();
    }
  }
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

template <int NP>
__global__ __launch_bounds__(128) void k_gather(GatherArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.K) return;
  float acc[NP];
  if (a.status[1] != 0) {
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = 0.0f;
  } else {
    gather_kernel_grads<NP>(j, a.ntx, a.tile_rects, a.ranges, a.vals, a.pair_grads, acc);
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) a.grads[(size_t)j * NP + i] = acc[i];
}

template <int C, int ORDER>
hipError_t launch_bwd(const BackwardArgs& a, hipStream_t s) {
  k_backward<C, ORDER><<<a.g.T, kThreads, 0, s>>>(a);
  return hipGetLastError();
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
  if (m.C == 1 && m.order == 0) return launch_bwd<1, 0>(a, s);
  if (m.C == 1 && m.order == 1) return launch_bwd<1, 1>(a, s);
  if (m.C == 3 && m.order == 0) return launch_bwd<3, 0>(a, s);
  return launch_bwd<3, 1>(a, s);
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
  const int blocks = (m.K + 127) / 128;
  const int NP = num_params(m.C, m.order);
  if (NP == 7) k_gather<7><<<blocks, 128, 0, s>>>(a);
  else if (NP == 9) k_gather<9><<<blocks, 128, 0, s>>>(a);  // (C, order) = (1, 1) or (3, 0)
  else k_gather<15><<<blocks, 128, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace smoe
