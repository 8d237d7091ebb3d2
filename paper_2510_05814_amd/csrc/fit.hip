// Fit-step kernels on gfx950 (Sec. VI-B: gradient descent with Adam on all kernel
// parameters, the centre learning rate decaying exponentially).
//
// A fit step runs three kernels (a fit's first step computes the render records first): the
// scatter of the (block, kernel) pairs into fixed-width block buckets, over each kernel's
// block rectangle computed from its model row (binning.hip), then
//   k_fit_tile: one wave per 16x16 block orders the block's bucket, renders the block
//     (image, D, squared error) and runs the backward over the same list while the
//     pixels' y, D and dL/dy are still in its registers -- the backward of a block needs
//     only that block's pixels, so nothing round-trips through HBM between the two;
//   k_adam_fit: per kernel, the sum of its block partials, Adam, re-materialization, and
//     the next step's render record.
// Cross-workgroup handoffs happen only at kernel boundaries: the 8 XCD L2 caches are not
// coherent with each other, so a device-scope fence per workgroup would cost more than a
// launch.  The step counter is read by every Adam workgroup and advanced by one: the
// scatter (the step's first kernel) copies it into a shadow status word that the later
// kernels read, so the single writer never races the readers.  A bucket overflow sets the
// step's flag (status word kStepFlags + parity of the step counter); Adam clears the next
// step's flag, which no kernel of this step reads.
#include "tile_math.h"

namespace smoe {
namespace {

struct FitTileArgs {
  Segs S;
  int shift;  // bucket entries: kernel id << shift | row of the entry's partial
  const float* __restrict__ records;
  int2* __restrict__ ranges;
  uint32_t* __restrict__ vals;
  uint32_t* __restrict__ vals_alt;
  int32_t* __restrict__ cursors;
  int32_t* __restrict__ status;
  int width;
  const float* __restrict__ target;
  float* __restrict__ image;  // null: the step's render is not stored
  float* __restrict__ denom;
  float* __restrict__ tile_loss;
  float* __restrict__ pair_grads;
};

template <int C, int ORDER, bool RBF, int TRUNC>
__global__ __launch_bounds__(kWave) void k_fit_tile(FitTileArgs a) {
  constexpr int LDS_FLOATS = kChunk * record_stride(C, ORDER);
  static_assert(LDS_FLOATS >= 64, "the rank sort's scratch lives in the record buffer");
  __shared__ float4 srec[LDS_FLOATS / 4];
  __shared__ uint32_t s_ent[kChunk];  // the entries of the chunk being staged
  const int tile = xcd_block(blockIdx.x, a.S.T);
  const int t0 = a.status[kStepShadow];
  // The bucket's fill count; the cursor is then reset for the next step's scatter (the store
  // depends on the loaded value, so it cannot overtake the load).
  const int cnt = a.cursors[tile];
  if (threadIdx.x == 0 && cnt >= 0) a.cursors[tile] = 0;
  if (a.status[kStepFlags + (t0 & 1)] != 0) {
    // Some bucket overflowed: nothing is rendered or updated this step.  The status words
    // report the storage a step needs (blocks x longest bucket).
    if (threadIdx.x == 0 && cnt > a.width) {
      atomicMax(&a.status[2], cnt);
      atomicMax(&a.status[0], (int)min((long long)cnt * a.S.T, (long long)INT32_MAX));
      a.status[1] = 1;
    }
    return;
  }
  const int2 rg = make_int2(tile * a.width, tile * a.width + cnt);
  if (threadIdx.x == 0) a.ranges[tile] = rg;  // the gradient gather reads the list back
  const SegGrid sg = seg_of_tile(a.S, tile);
  // MSE of this raster: dL/dy = 2 (y - t) / (W H C); its squared errors are stored already
  // divided by W H C, so that the sum over all blocks is the sum of the rasters' MSEs.
  const float inv_n2 = 2.0f / ((float)sg.W * (float)sg.H * (float)C);
  const float inv_n = 1.0f / ((float)sg.W * (float)sg.H * (float)C);
  // Order the bucket (the scatter appended in arbitrary order).  A bucket of one chunk is
  // ranked in registers and kept in LDS for the forward's staging.
  constexpr int run = LDS_FLOATS >= 1024 ? 1024 : (LDS_FLOATS >= 512 ? 512 : 256);
  if (rg.y - rg.x <= kChunk) {
    rank_sort64(a.vals + rg.x, rg.y - rg.x, reinterpret_cast<uint32_t*>(srec), s_ent);
  } else {
    sort_bucket(a.vals + rg.x, a.vals_alt + rg.x, rg.y - rg.x, reinterpret_cast<uint32_t*>(srec),
                run);
  }

  const PixelCoords px = lane_pixels(sg, tile - sg.tile_offset);
  float D[kRows], N[kRows][C];
  uint64_t live = 0;
  forward_accumulate<C, ORDER, TRUNC>(px, a.S.r2, a.S.cut_scale, a.S.cut_offset, a.records,
                                      a.vals, a.shift, rg, srec, D, N, live, s_ent);

  PixelSeed<C> sd;
  float err = 0.0f;
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
      const bool cov = D[i] > 0.0f;
      // 1/D by v_rcp_f32 (1 ulp); y = N / D refined from it, as in the render
      const float invD = RBF ? 1.0f : (cov ? __builtin_amdgcn_rcpf(D[i]) : 0.0f);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        // Eq. (2)-(4): y = N / D; Eq. (1): y = N
        const float yc = RBF ? N[i][c] : (cov ? div_refined(N[i][c], D[i], invD) : 0.0f);
        if (a.image) a.image[p * C + c] = yc;
        const float d = yc - a.target[p * C + c];
        err = __builtin_fmaf(d, d, err);
        if (cov) {
          sd.g[i][c] = d * inv_n2;
          if (!RBF) sd.gy[i] = __builtin_fmaf(sd.g[i][c], yc, sd.gy[i]);
        }
      }
      if (a.image) a.denom[p] = D[i];
      sd.valid[i] = cov;
      sd.invD[i] = invD;
    }
  }
  for (int off = 32; off > 0; off >>= 1) err += __shfl_xor(err, off);
  if (threadIdx.x == 0) a.tile_loss[tile] = err * inv_n;

  // each partial row goes to the row its entry names, where Adam reads it
  backward_accumulate<C, ORDER>(px, a.S.r2, a.records, a.vals, a.shift, true, rg, srec, true,
                                live, sd, a.pair_grads, a.S.K);
}

struct AdamFitArgs {
  Segs S;
  int shift;  // bucket entries: kernel id << shift | row of the partial (k_scatter_fixed)
  const int4* __restrict__ tile_rects;  // the step's block rectangles (from its scatter)
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  const float* __restrict__ pair_grads;
  const float* __restrict__ tile_loss;  // per-block squared errors / (W H C)
  int32_t* __restrict__ status;
  StepScalarsArgs step;
  float* __restrict__ raw;
  float* __restrict__ m;
  float* __restrict__ v;
  float* __restrict__ model;
  float* __restrict__ grads;
  float* __restrict__ records;
};


// Fit-step Adam fused with the re-materialization.  16 lanes per kernel: lane i owns raw
// parameter i -- its gradient (the sum of the kernel's block partials), Adam with the group's
// learning rate, the re-materialized value -- and writes field i of the new render record
// (the next step's scatter derives the block rectangle from the new model row).  Block 0
// also reduces the per-block squared errors into the loss.  After an overflow the
// parameters stay as they are, and the records are rewritten from them unchanged.
constexpr int kAdamThreads = 256;
// (held to 64 VGPRs: 8 waves per SIMD to overlap the gather's loads)
template <int C, int ORDER>
__global__ __launch_bounds__(kAdamThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_adam_fit(AdamFitArgs f) {
  constexpr int NP = num_params(C, ORDER);
  constexpr int NE = expert_floats(C, ORDER);
  constexpr int RS = record_stride(C, ORDER);
  __shared__ float s_red[kAdamThreads / 64];
  const smoe_adam_config& ad = f.step.adam;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = gid >> 4, i = gid & 15;
  const bool live = j < f.S.K;
  const size_t e = (size_t)j * NP + i;
  // Every load that depends on no other is issued before the first wait: the status words
  // (the completed steps, copied by this step's scatter, and both overflow flags), the step's
  // Adam scalars (written by the scatter), the kernel's block rectangle and Adam's state.
  const int t0 = f.status[kStepShadow];
  const int flag0 = f.status[kStepFlags], flag1 = f.status[kStepFlags + 1];
  const float lr_mu = f.step.scalars[0], bc1 = f.step.scalars[1], bc2 = f.step.scalars[2];
  int4 rc = make_int4(0, 0, -1, -1);
  float m0 = 0.0f, v0 = 0.0f, raw0 = 0.0f;
  if (live) {
    rc = f.tile_rects[j];
    if (i < NP) {
      m0 = f.m[e];
      v0 = f.v[e];
      raw0 = f.raw[e];
    }
  }
  const bool skip = ((t0 & 1) ? flag1 : flag0) != 0;
  if (blockIdx.x == 0 && !skip) {
    // Loss: the whole workgroup sums the per-block squared errors in a fixed order, four
    // independent float4 streams per thread so that the loads overlap.
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const int T4 = f.S.T >> 2;
    const float4* tl4 = reinterpret_cast<const float4*>(f.tile_loss);
    for (int q = threadIdx.x; q < T4; q += 4 * kAdamThreads) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int qq = q + u * kAdamThreads;
        if (qq < T4) {
          const float4 v = tl4[qq];
          acc[u] += (v.x + v.y) + (v.z + v.w);
        }
      }
    }
    for (int t = (T4 << 2) + threadIdx.x; t < f.S.T; t += kAdamThreads) acc[0] += f.tile_loss[t];
    float tot = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
      float sum = 0.0f;
      for (int w = 0; w < kAdamThreads / 64; ++w) sum += s_red[w];
      const float loss = sum;
      if (f.step.loss_out) f.step.loss_out[0] = loss;
      if (f.step.loss_history && t0 < f.step.max_steps) f.step.loss_history[t0] = loss;
    }
  }

  const SegGrid sg = seg_of_kernel(f.S, live ? j : 0);
  float pm = 0.0f;  // materialized value of parameter i after the step
  if (live && skip && i < NP) pm = f.model[e];
  const bool upd = live && !skip && i < NP;
  // Every lane takes part in the gather's row reduction and the finishing shuffles; the
  // expert slopes are those of the raw row (the render record this step used holds the same
  // numbers).
  const float gi = finish_gradient<C, ORDER, 6>(
      gather_param_fit<NP>(j, live && !skip, sg, rc, f.S.K, f.ranges, f.vals, f.pair_grads,
                           f.shift),
      live && !skip, raw0);
  if (upd) {
    const float lr = i < 2 ? lr_mu : (i < 5 ? ad.lr_chol : (i == 5 ? ad.lr_rho : ad.lr_expert));
    const float mi = ad.beta1 * m0 + (1.0f - ad.beta1) * gi;
    const float vi = ad.beta2 * v0 + (1.0f - ad.beta2) * gi * gi;
    f.m[e] = mi;
    f.v[e] = vi;
    const float p = raw0 - lr * (mi / bc1) / (sqrtf(vi / bc2) + ad.eps);
    f.raw[e] = p;
    pm = (i == 2 || i == 4) ? expf(p) : p;
    f.model[e] = pm;
    if (f.grads) f.grads[e] = gi;
  }
  // The kernel's new row, shared inside its group of 16 lanes.
  const float mux = __shfl(pm, 0, 16), muy = __shfl(pm, 1, 16), l11 = __shfl(pm, 2, 16);
  const float l21 = __shfl(pm, 3, 16), l22 = __shfl(pm, 4, 16), rho = __shfl(pm, 5, 16);
  const float prev = __shfl_up(pm, 1, 16);  // parameter i - 1
  // A row with a NaN or infinite parameter covers no block in the next step (it takes part
  // nowhere) and sets the non-finite status word.
  const unsigned long long nf = __ballot(i < NP && !__builtin_isfinite(pm));
  const bool row_nonfinite = ((nf >> (threadIdx.x & 48)) & 0xFFFFull) != 0;
  if (live) {
    if (i < RS) {
      const float i22 = 1.0f / l22;
      float fld;
      if (i == 0) fld = mux;
      else if (i == 1) fld = muy;
      else if (i == 2) fld = 1.0f / l11;
      else if (i == 3) fld = l21;
      else if (i == 4) fld = i22;
      else if (i == 5) fld = rho * kLog2e;
      else if (i == 6) fld = l21 * i22;
      else if (i < kRecExpert + NE) fld = prev;
      else fld = 0.0f;
      f.records[(size_t)j * RS + i] = fld;
    }
    if (i == 0 && row_nonfinite) f.status[kNonfinite] = 1;
  }
  // The counter itself is written once; every workgroup read the shadow copy instead.  The
  // next step's overflow flag is cleared here: no kernel of this step reads it.
  if (blockIdx.x == 0 && threadIdx.x == 0 && !skip) {
    f.step.step[0] = t0 + 1;
    f.status[kStepFlags + ((t0 + 1) & 1)] = 0;
  }
}

// Reporting: the loss of each raster of the last fit step (one workgroup per segment sums
// its blocks' normalised squared errors in a fixed order).
__global__ __launch_bounds__(256) void k_segment_losses(Segs S, const float* __restrict__ tile_loss,
                                                        float* __restrict__ out) {
  __shared__ float s_red[4];
  const smoe_segment seg = S.tab ? S.tab[blockIdx.x] : S.one;
  const int T0 = seg.tile_offset;
  const int Ts = blocks_across(seg.width, seg.origin_x) * blocks_across(seg.height, seg.origin_y);
  float acc = 0.0f;
  for (int t = threadIdx.x; t < Ts; t += 256) acc += tile_loss[T0 + t];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

__global__ __launch_bounds__(128) void k_materialize(int n_rows, int NP,
                                                     const float* __restrict__ raw,
                                                     float* __restrict__ model) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows * NP) return;
  const int k = i % NP;
  const float x = raw[i];
  model[i] = (k == 2 || k == 4) ? expf(x) : x;
}

}  // namespace

hipError_t launch_fit_tile(const smoe_fit_state& st, const Segs& S, int width, int shift,
                           const float* target, hipStream_t s) {
  const smoe_bins& b = st.bins;
  FitTileArgs a{S,        shift,     b.records, reinterpret_cast<int2*>(b.ranges),
                b.vals,   b.vals_alt, b.tile_counts, b.status, width,
                target,   st.write_render ? st.image : nullptr,
                st.write_render ? st.denom : nullptr,
                b.tile_loss, b.pair_grads};
  with_shape(st.C, st.order, S, [&](auto sh) {
    using T = decltype(sh);
    k_fit_tile<T::C, T::ORDER, T::RBF, T::TRUNC><<<S.T, kWave, 0, s>>>(a);
  });
  return hipGetLastError();
}

hipError_t launch_adam_fit(const smoe_fit_state& st, const Segs& S, int shift, float* loss_out,
                           hipStream_t s) {
  const smoe_bins& b = st.bins;
  AdamFitArgs f{S,
                shift,
                reinterpret_cast<const int4*>(b.tile_rects),
                reinterpret_cast<const int2*>(b.ranges),
                b.vals,
                b.pair_grads,
                b.tile_loss,
                b.status,
                make_step_scalars_args(st, loss_out),
                st.raw,
                st.adam_m,
                st.adam_v,
                st.model,
                st.grads,
                b.records};
  // at least one workgroup, so that the loss and the step counter advance even for K = 0
  const int blocks = max(1, (int)(((long long)S.K * 16 + kAdamThreads - 1) / kAdamThreads));
  if (st.C == 1 && st.order == 0) k_adam_fit<1, 0><<<blocks, kAdamThreads, 0, s>>>(f);
  else if (st.C == 1 && st.order == 1) k_adam_fit<1, 1><<<blocks, kAdamThreads, 0, s>>>(f);
  else if (st.C == 3 && st.order == 0) k_adam_fit<3, 0><<<blocks, kAdamThreads, 0, s>>>(f);
  else k_adam_fit<3, 1><<<blocks, kAdamThreads, 0, s>>>(f);
  return hipGetLastError();
}

hipError_t launch_segment_losses(const Segs& S, const smoe_bins& b, float* out, hipStream_t s) {
  k_segment_losses<<<S.tab ? S.n : 1, 256, 0, s>>>(S, b.tile_loss, out);
  return hipGetLastError();
}

hipError_t launch_materialize(int K, int C, int order, const float* raw, float* model,
                              hipStream_t s) {
  const int NP = num_params(C, order);
  const long long n = (long long)K * NP;
  if (n == 0) return hipSuccess;
  k_materialize<<<(int)((n + 127) / 128), 128, 0, s>>>(K, NP, raw, model);
  return hipGetLastError();
}

}  // namespace smoe
