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
// Work split: one wave per 16x16 block; lane l owns column l & 15 and the four rows
// (l >> 4) + 4i, i = 0..3, so the column-only terms (dx, z1, l21 z1, z1^2) of the exact
// truncation test are computed once per kernel for four pixels.  The block's kernel list
// is staged through LDS in chunks.  Per kernel the wave's 16 accumulators (6 + 3C <= 15
// used) are summed over the 64 lanes by a transposed butterfly (cross-half swaps, then
// DPP), which leaves lane 4v holding the total of accumulator v; those lanes write the
// per-(block, kernel) partial row.  A second pass sums each kernel's partial rows over its
// blocks in row-major block order.  Every order is fixed: gradients are bitwise
// reproducible and no atomics are used.
#include "smoe_internal.h"

namespace smoe {
namespace {

constexpr int kThreads = 64;     // one wave per block
constexpr int kChunk = 64;       // records staged in LDS per chunk
constexpr int kRows = kTile * kTile / kThreads;  // pixels per lane (4)

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

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Transposed wave reduction of 16 values: on return lane l holds the sum over all 64 lanes
// of v[(l >> 2) & 15].  Each stage pairs every lane with one whose index differs in the next
// bit (5, 4, 3, 2); a lane keeps the half of its values selected by that bit and adds the
// partner's copy of the same half, halving the values per lane.  Bits 1 and 0 are then a
// plain butterfly.  About 40 instructions for 16 sums instead of 6 per sum.
__device__ __forceinline__ float wave_reduce16_transposed(float (&v)[16]) {
  const int lane = threadIdx.x & 63;
  // bit 5: v_permlane32_swap exchanges lanes 32-63 of its first operand with lanes 0-31 of
  // its second, so (a + b) of the two results holds sum(v[i]) in the low half and
  // sum(v[i + 8]) in the high half.
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]),
                                                    false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // bit 4: v_permlane16_swap exchanges the odd 16-lane rows of its first operand with the
  // even rows of its second.
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]),
                                                    false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // bit 3: DPP row_ror:8 pairs lane l with l ^ 8 inside each row of 16.
  const bool b3 = (lane & 8) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b3 ? v[i + 2] : v[i];
    const float send = b3 ? v[i] : v[i + 2];
    v[i] = keep + dpp<0x128>(send);
  }
  // bit 2: DPP row_half_mirror pairs lane l with 7 - l inside each group of 8.
  const bool b2 = (lane & 4) != 0;
  {
    const float keep = b2 ? v[1] : v[0];
    const float send = b2 ? v[0] : v[1];
    v[0] = keep + dpp<0x141>(send);
  }
  v[0] += dpp<0x4E>(v[0]);  // quad_perm [2, 3, 0, 1]: bit 1
  v[0] += dpp<0xB1>(v[0]);  // quad_perm [1, 0, 3, 2]: bit 0
  return v[0];
}

template <int C, int ORDER>
__global__ __launch_bounds__(kThreads) void k_backward(BackwardArgs a) {
  constexpr int RS = record_stride(C, ORDER);
  constexpr int NP = num_params(C, ORDER);
  static_assert(NP <= 16, "16 accumulators per kernel");
  __shared__ float4 srec[kChunk * RS / 4];

  const int lane = threadIdx.x;
  const int tile = xcd_block(blockIdx.x, a.g.T);
  const int tx = tile % a.g.ntx, ty = tile / a.g.ntx;
  const int u = tx * kTile + (lane & 15);
  const float x = sample_coord(u, a.g.ox, a.g.inv_s);
  const float r2 = a.g.r2;
  const int2 rg = a.ranges[tile];

  // Per-pixel adjoint seeds of the lane's four pixels.
  float yv[kRows], invD[kRows], gyv[kRows], g[kRows][C];
  bool valid[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int v = ty * kTile + (lane >> 4) + 4 * i;
    yv[i] = sample_coord(v, a.g.oy, a.g.inv_s);
    valid[i] = false;
    invD[i] = 0.0f;
    gyv[i] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) g[i][c] = 0.0f;
    if (u < a.g.W && v < a.g.H) {
      const size_t p = (size_t)v * a.g.W + u;
      const float D = a.denom[p];
      if (D > 0.0f) {
        valid[i] = true;
        invD[i] = 1.0f / D;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const float yc = a.image[p * C + c];
          g[i][c] = a.target ? (yc - a.target[p * C + c]) * a.inv_n2 : a.grad_image[p * C + c];
          gyv[i] = __builtin_fmaf(g[i][c], yc, gyv[i]);
        }
      }
    }
  }

  for (int base = rg.x; base < rg.y; base += kChunk) {
    const int n = min(kChunk, rg.y - base);
    __syncthreads();
    constexpr int Q = RS / 4;
    for (int i = lane; i < n * Q; i += kThreads) {
      const int k = i / Q, c = i - k * Q;
      srec[i] = reinterpret_cast<const float4*>(a.records + (size_t)a.vals[base + k] * RS)[c];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const float* r = reinterpret_cast<const float*>(&srec[k * Q]);
      float acc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
      // column terms of the truncation test, shared by the lane's four pixels
      const float dx = x - r[0];
      const float z1 = dx * r[2];
      const float tt = r[3] * z1;
      const float zz1 = z1 * z1;
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        const float dy = yv[i] - r[1];
        const float w_ = dy - tt;
        const float z2 = w_ * r[4];
        const float q = zz1 + z2 * z2;
        if (valid[i] && q <= r2) {
          const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(q, -0.5f * kLog2e, r[5]));
          const float w = e * invD[i];
          float Gs = -gyv[i];
          float ex = 0.0f, ey = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            float m = r[kRecExpert + c];
            if (ORDER == 1) {
              m = __builtin_fmaf(r[kRecExpert + C + c], dx, m);
              m = __builtin_fmaf(r[kRecExpert + 2 * C + c], dy, m);
            }
            Gs = __builtin_fmaf(g[i][c], m, Gs);
            const float gw = g[i][c] * w;
            acc[6 + c] += gw;
            if (ORDER == 1) {
              acc[6 + C + c] = __builtin_fmaf(gw, dx, acc[6 + C + c]);
              acc[6 + 2 * C + c] = __builtin_fmaf(gw, dy, acc[6 + 2 * C + c]);
              ex = __builtin_fmaf(gw, r[kRecExpert + C + c], ex);
              ey = __builtin_fmaf(gw, r[kRecExpert + 2 * C + c], ey);
            }
          }
          const float Hh = w * Gs;
          const float bz2 = -Hh * z2;
          const float bz1 = __builtin_fmaf(-bz2, r[6], -Hh * z1);
          acc[0] -= __builtin_fmaf(bz1, r[2], ex);
          acc[1] -= __builtin_fmaf(bz2, r[4], ey);
          acc[2] = __builtin_fmaf(-bz1, z1, acc[2]);
          acc[3] = __builtin_fmaf(-bz2 * z1, r[4], acc[3]);
          acc[4] = __builtin_fmaf(-bz2, z2, acc[4]);
          acc[5] += Hh;
        }
      }
      const float tot = wave_reduce16_transposed(acc);
      const int idx = lane >> 2;
      if ((lane & 3) == 0 && idx < NP) a.pair_grads[(size_t)(base + k) * NP + idx] = tot;
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
  const int blocks = (int)(((long long)m.K * 16 + 255) / 256);
  const int NP = num_params(m.C, m.order);
  if (NP == 7) k_gather<7><<<blocks, 256, 0, s>>>(a);
  else if (NP == 9) k_gather<9><<<blocks, 256, 0, s>>>(a);  // (C, order) = (1, 1) or (3, 0)
  else k_gather<15><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace smoe
