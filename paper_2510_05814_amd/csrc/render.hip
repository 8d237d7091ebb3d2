// Forward rasterization of the SMoE regression (Eq. 3-5) on gfx950: the standalone render.
//
// One wave (64 lanes) per 16x16 block (lane layout in tile_math.h).  The block's kernel
// list is staged through LDS in chunks of 64 render records (coalesced float4 loads); the
// wave reads each record with a uniform LDS address (a broadcast) and accumulates, in FP32
// registers, the gate denominator D = sum_j pi_j K_j(x) and the numerators
// N_c = sum_j pi_j K_j(x) m_jc(x) of each pixel in list order (increasing kernel id);
// y_c = N_c / D.  No MFMA: there is no dense contraction here, the work is FP32 VALU plus
// one v_exp_f32 per participating pair.
//
// Long lists (more than kSplitMin entries, which only very wide kernels produce) are split
// over the four waves of a workgroup instead (k_render_wide): wave w accumulates the w-th
// contiguous quarter of the list, and wave 0 adds the four partial sums in wave order -- a
// fixed order, so the render stays deterministic.  Every block is rendered by exactly one of
// the two kernels.
//
// Optional fused squared error against a target: each block writes its sum of squared
// errors to tile_loss[block]; launch_loss_reduce() then reduces those in a fixed order.
#include "tile_math.h"

namespace smoe {
namespace {

struct RenderArgs {
  Segs S;
  const float* __restrict__ records;
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  float* __restrict__ image;
  float* __restrict__ denom;
  const float* __restrict__ target;
  float* __restrict__ tile_loss;
  const int32_t* __restrict__ status;  // the binning's status words (word 2: longest list)
};

// Blocks whose list is longer than this go to k_render_wide.
constexpr int kSplitMin = 2 * kChunk;
constexpr int kSplitWaves = 4;

// Writes the block's pixels (y from N and D, Eq. 2-4 or Eq. 1) and its squared error.
template <int C, bool RBF>
__device__ __forceinline__ void render_epilogue(const RenderArgs& a, const SegGrid& sg,
                                                const PixelCoords& px, int tile,
                                                const float (&D)[kRows],
                                                const float (&N)[kRows][C]) {
  float err = 0.0f;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int v = px.v0 + 4 * i;
    if (in_raster(px.u, v, sg)) {
      const size_t p = (size_t)sg.pixel_offset + (size_t)v * sg.W + px.u;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        // Eq. (2)-(4): y = N / D, refined from v_rcp_f32(D) exactly as the fit step's render;
        // Eq. (1): y = N
        const float yc =
            RBF ? N[i][c]
                : ((D[i] > 0.0f) ? div_refined(N[i][c], D[i], __builtin_amdgcn_rcpf(D[i])) : 0.0f);
        a.image[p * C + c] = yc;
        if (a.target) {
          const float d = yc - a.target[p * C + c];
          err = __builtin_fmaf(d, d, err);
        }
      }
      if (a.denom) a.denom[p] = D[i];
    }
  }
  if (a.tile_loss) {
    for (int off = 32; off > 0; off >>= 1) err += __shfl_xor(err, off);
    if ((threadIdx.x & 63) == 0) a.tile_loss[tile] = err;
  }
}

template <int C, int ORDER, bool RBF, int TRUNC>
__global__ __launch_bounds__(kWave) void k_render(RenderArgs a) {
  __shared__ float4 srec[kChunk * record_stride(C, ORDER) / 4];
  const int tile = xcd_block(blockIdx.x, a.S.T);
  const int2 rg = a.ranges[tile];
  if (rg.y - rg.x > kSplitMin) return;  // a long list: k_render_wide renders this block
  const SegGrid sg = seg_of_tile(a.S, tile);
  const PixelCoords px = lane_pixels(sg, tile - sg.tile_offset);
  float D[kRows], N[kRows][C];
  uint64_t live;
  forward_accumulate<C, ORDER, TRUNC>(px, a.S.r2, a.S.cut_scale, a.S.cut_offset, a.records,
                                      a.vals, 0, rg, srec, D, N, live);
  render_epilogue<C, RBF>(a, sg, px, tile, D, N);
}

// Four waves per block for lists longer than kSplitMin.  Each wave stages its own records
// in its own LDS region; within a wave, LDS stores and loads execute in program order, so
// the staging needs no workgroup barrier (the waves' chunk counts differ).  A workgroup
// walks the blocks with a grid stride (at most kWideGroups workgroups); a raster whose
// longest list (status word 2 of its binning) is short costs only the launch.  Every
// decision in the walk is the same for the four waves, so each barrier is reached by all
// of them.
constexpr int kWideGroups = 1024;

template <int C, int ORDER, bool RBF, int TRUNC>
__device__ __forceinline__ void render_wide_block(const RenderArgs& a, int tile, int2 rg,
                                                  float4 (*srec)[kChunk * record_stride(C, ORDER) / 4],
                                                  float (*part)[kRows * (1 + C)][kWave]) {
  constexpr int RS = record_stride(C, ORDER);
  constexpr int Q = RS / 4;
  const int len = rg.y - rg.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const SegGrid sg = seg_of_tile(a.S, tile);
  const PixelCoords px = lane_pixels(sg, tile - sg.tile_offset);
  const int per = (len + kSplitWaves - 1) / kSplitWaves;
  const int b = rg.x + min(len, wv * per), e = rg.x + min(len, (wv + 1) * per);
  float D[kRows], N[kRows][C];
  zero_sums<C>(D, N);
  const float cut_scale = in_vgpr(a.S.cut_scale), cut_offset = in_vgpr(a.S.cut_offset);
  float4* my = srec[wv];
  for (int base = b; base < e; base += kChunk) {
    const int n = min(kChunk, e - base);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < n * Q; i += kWave) {
      const int k = i / Q, c = i - k * Q;
      my[i] = reinterpret_cast<const float4*>(a.records + (size_t)a.vals[base + k] * RS)[c];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int k = 0; k < n; ++k)
      forward_entry<C, ORDER, TRUNC>(px, a.S.r2, cut_scale, cut_offset,
                                     reinterpret_cast<const float*>(&my[k * Q]), D, N);
  }
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      part[wv - 1][i * (1 + C)][lane] = D[i];
#pragma unroll
      for (int c = 0; c < C; ++c) part[wv - 1][i * (1 + C) + 1 + c][lane] = N[i][c];
    }
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int w = 0; w < kSplitWaves - 1; ++w) {
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        D[i] += part[w][i * (1 + C)][lane];
#pragma unroll
        for (int c = 0; c < C; ++c) N[i][c] += part[w][i * (1 + C) + 1 + c][lane];
      }
    }
    render_epilogue<C, RBF>(a, sg, px, tile, D, N);
  }
  __syncthreads();  // part is reused by the next block of the walk
}

template <int C, int ORDER, bool RBF, int TRUNC>
__global__ __launch_bounds__(kSplitWaves * kWave) void k_render_wide(RenderArgs a) {
  __shared__ float4 srec[kSplitWaves][kChunk * record_stride(C, ORDER) / 4];
  __shared__ float part[kSplitWaves - 1][kRows * (1 + C)][kWave];
  // the binning recorded the longest list: without a long one there is nothing to walk
  if (a.status[2] <= kSplitMin) return;
  for (int tile = blockIdx.x; tile < a.S.T; tile += gridDim.x) {
    const int2 rg = a.ranges[tile];
    if (rg.y - rg.x <= kSplitMin) continue;  // k_render renders this block
    render_wide_block<C, ORDER, RBF, TRUNC>(a, tile, rg, srec, part);
  }
}

// One workgroup: loss = inv_n * sum of the per-block partials, in a fixed order.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_loss_reduce(const float* __restrict__ part,
                                                                int T, float inv_n,
                                                                float* __restrict__ out) {
  __shared__ float s[kReduceThreads / 64];
  float acc = 0.0f;
  for (int i = threadIdx.x; i < T; i += kReduceThreads) acc += part[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < kReduceThreads / 64; ++w) t += s[w];
    out[0] = t * inv_n;
  }
}

// Diagnostic: per block, the tested (pixel, kernel) pairs of in-image pixels and those with
// q <= r^2, added atomically into out2 = (tested, active).
constexpr int kStatThreads = kTilePixels;
__global__ __launch_bounds__(kStatThreads) void k_pair_stats(Segs S, const float* __restrict__ records,
                                                             int rs, const int2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ vals,
                                                             unsigned long long* __restrict__ out2) {
  __shared__ unsigned long long s_act[kStatThreads / 64];
  __shared__ unsigned long long s_cnt[kStatThreads / 64];
  const int tile = blockIdx.x;
  const SegGrid g = seg_of_tile(S, tile);
  const int lt = tile - g.tile_offset;
  const int tx = lt % g.ntx, ty = lt / g.ntx;
  const int u = kTile * (g.bx0 + tx) - g.ox + (threadIdx.x & 15);
  const int v = kTile * (g.by0 + ty) - g.oy + (threadIdx.x >> 4);
  const bool inside = (unsigned)u < (unsigned)g.W && (unsigned)v < (unsigned)g.H;
  const float x = sample_coord(u, g.ox, g.inv_s);
  const float y = sample_coord(v, g.oy, g.inv_s);
  const int2 rg = ranges[tile];
  unsigned long long act = 0;
  for (int i = rg.x; i < rg.y && inside; ++i) {
    const float* r = records + (size_t)vals[i] * rs;
    const float dx = x - r[0];
    const float dy = y - r[1];
    const float z1 = dx * r[2];
    const float tt = r[3] * z1;
    const float w = dy - tt;
    const float z2 = w * r[4];
    const float q = z1 * z1 + z2 * z2;
    act += (q <= S.r2) ? 1ull : 0ull;
  }
  unsigned long long cnt = inside ? 1ull : 0ull;
  for (int off = 32; off > 0; off >>= 1) {
    act += __shfl_xor(act, off);
    cnt += __shfl_xor(cnt, off);
  }
  if ((threadIdx.x & 63) == 0) {
    s_act[threadIdx.x >> 6] = act;
    s_cnt[threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long px = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    atomicAdd(&out2[0], px * (unsigned long long)(rg.y - rg.x));
    atomicAdd(&out2[1], s_act[0] + s_act[1] + s_act[2] + s_act[3]);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_render(int C, int order, const Segs& S, const smoe_bins& b, float* image,
                         float* denom, const float* target, hipStream_t s) {
  RenderArgs a{S,
               b.records,
               reinterpret_cast<const int2*>(b.ranges),
               b.vals,
               image,
               denom,
               target,
               target ? b.tile_loss : nullptr,
               b.status};
  with_shape(C, order, S, [&](auto sh) {
    using T = decltype(sh);
    k_render<T::C, T::ORDER, T::RBF, T::TRUNC><<<S.T, kWave, 0, s>>>(a);
    k_render_wide<T::C, T::ORDER, T::RBF, T::TRUNC>
        <<<min(S.T, kWideGroups), kSplitWaves * kWave, 0, s>>>(a);
  });
  return hipGetLastError();
}

hipError_t launch_pair_stats(const Segs& S, const smoe_bins& b, uint64_t* out2, hipStream_t s) {
  k_zero_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long*>(out2), 2);
  k_pair_stats<<<S.T, kStatThreads, 0, s>>>(S, b.records, b.record_stride,
                                            reinterpret_cast<const int2*>(b.ranges), b.vals,
                                            reinterpret_cast<unsigned long long*>(out2));
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const smoe_bins& b, int T, float inv_n, float* loss_out,
                              hipStream_t s) {
  k_loss_reduce<<<1, kReduceThreads, 0, s>>>(b.tile_loss, T, inv_n, loss_out);
  return hipGetLastError();
}

}  // namespace smoe
