// Fit-step kernels on gfx950: raw -> materialized parameters, the per-step scalars (loss,
// step counter, learning rates, bias corrections), and the fused per-kernel
// "gather block partials -> Adam -> re-materialize" update (Sec. VI-B: Adam, centre rate
// decaying exponentially).  Element-wise and HBM-bound.
#include "smoe_internal.h"

namespace smoe {
namespace {

// Scalars written by k_step_begin and read by k_adam (same stream, so ordered):
//   [0] centre learning rate of this step   [1] 1 - beta1^t   [2] 1 - beta2^t
//   [3] 1 when this step must change nothing (pair-capacity overflow)
constexpr int kSkip = 3;

__global__ __launch_bounds__(128) void k_materialize(int n_rows, int NP,
                                                     const float* __restrict__ raw,
                                                     float* __restrict__ model) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows * NP) return;
  const int k = i % NP;
  const float x = raw[i];
  model[i] = (k == 2 || k == 4) ? expf(x) : x;
}

constexpr int kReduceThreads = 1024;

struct StepBeginArgs {
  const float* __restrict__ tile_loss;
  int T;
  float inv_n;
  const int32_t* __restrict__ status;
  int32_t* __restrict__ step;
  float* __restrict__ scalars;
  float* __restrict__ loss_out;
  float* __restrict__ loss_history;
  int max_steps;
  smoe_adam_config adam;
};

// One workgroup: loss = inv_n * sum of the block partials (fixed order), then the step's
// scalars, then the step counter.  After an overflow nothing advances.
__global__ __launch_bounds__(kReduceThreads) void k_step_begin(StepBeginArgs a) {
  __shared__ float s[kReduceThreads / 64];
  float acc = 0.0f;
  for (int i = threadIdx.x; i < a.T; i += kReduceThreads) acc += a.tile_loss[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  float tot = 0.0f;
  for (int w = 0; w < kReduceThreads / 64; ++w) tot += s[w];
  const float loss = tot * a.inv_n;
  if (a.status[1] != 0) {
    a.scalars[kSkip] = 1.0f;
    return;
  }
  const int t0 = a.step[0];
  if (a.loss_out) a.loss_out[0] = loss;
  if (a.loss_history && t0 < a.max_steps) a.loss_history[t0] = loss;
  float lr_mu = a.adam.lr_mu;
  if (a.adam.total_steps > 0 && a.adam.lr_mu > 0.0f && a.adam.lr_mu_final > 0.0f)
    lr_mu = a.adam.lr_mu * powf(a.adam.lr_mu_final / a.adam.lr_mu,
                                (float)t0 / (float)a.adam.total_steps);
  a.scalars[0] = lr_mu;
  a.scalars[1] = 1.0f - powf(a.adam.beta1, (float)(t0 + 1));
  a.scalars[2] = 1.0f - powf(a.adam.beta2, (float)(t0 + 1));
  a.scalars[kSkip] = 0.0f;
  a.step[0] = t0 + 1;
}

struct AdamArgs {
  int K;
  int ntx;
  const int4* __restrict__ tile_rects;
  const int2* __restrict__ ranges;
  const uint32_t* __restrict__ vals;
  const float* __restrict__ pair_grads;
  const float* __restrict__ scalars;
  float* __restrict__ raw;
  float* __restrict__ m;
  float* __restrict__ v;
  float* __restrict__ model;
  float* __restrict__ grads;
  smoe_adam_config adam;
};

// 16 lanes per kernel, lane i owning raw parameter i: its gradient (the sum of the
// kernel's block partials), Adam with the group's learning rate, and the re-materialized
// value.  Rows are read and written as contiguous 4*NP-byte runs.
template <int NP>
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = gid >> 4, i = gid & 15;
  if (j >= a.K || a.scalars[kSkip] != 0.0f) return;
  const float gi = gather_param<NP>(j, i, a.ntx, a.tile_rects, a.ranges, a.vals, a.pair_grads);
  if (i >= NP) return;
  const float lr = i < 2 ? a.scalars[0]
                         : (i < 5 ? a.adam.lr_chol : (i == 5 ? a.adam.lr_rho : a.adam.lr_expert));
  const float b1 = a.adam.beta1, b2 = a.adam.beta2;
  const size_t e = (size_t)j * NP + i;
  const float mi = b1 * a.m[e] + (1.0f - b1) * gi;
  const float vi = b2 * a.v[e] + (1.0f - b2) * gi * gi;
  a.m[e] = mi;
  a.v[e] = vi;
  const float p = a.raw[e] - lr * (mi / a.scalars[1]) / (sqrtf(vi / a.scalars[2]) + a.adam.eps);
  a.raw[e] = p;
  a.model[e] = (i == 2 || i == 4) ? expf(p) : p;
  if (a.grads) a.grads[e] = gi;
}

}  // namespace

hipError_t launch_materialize(int K, int C, int order, const float* raw, float* model,
                              hipStream_t s) {
  const int NP = num_params(C, order);
  const long long n = (long long)K * NP;
  if (n == 0) return hipSuccess;
  k_materialize<<<(int)((n + 127) / 128), 128, 0, s>>>(K, NP, raw, model);
  return hipGetLastError();
}

hipError_t launch_step_begin(const smoe_fit_state& st, const GridArgs& g, float inv_n,
                             float* loss_out, hipStream_t s) {
  StepBeginArgs a{st.bins.tile_loss, g.T,           inv_n,        st.bins.status,
                  st.step,           st.scalars,    loss_out,     st.loss_history,
                  st.max_steps,      st.adam};
  k_step_begin<<<1, kReduceThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_adam(const smoe_fit_state& st, const GridArgs& g, hipStream_t s) {
  if (st.K == 0) return hipSuccess;
  AdamArgs a{st.K,
             g.ntx,
             reinterpret_cast<const int4*>(st.bins.tile_rects),
             reinterpret_cast<const int2*>(st.bins.ranges),
             st.bins.vals,
             st.bins.pair_grads,
             st.scalars,
             st.raw,
             st.adam_m,
             st.adam_v,
             st.model,
             st.grads,
             st.adam};
  const int blocks = (int)(((long long)st.K * 16 + 255) / 256);
  const int NP = num_params(st.C, st.order);
  if (NP == 7) k_adam<7><<<blocks, 256, 0, s>>>(a);
  else if (NP == 9) k_adam<9><<<blocks, 256, 0, s>>>(a);  // (C, order) = (1, 1) or (3, 0)
  else k_adam<15><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace smoe
