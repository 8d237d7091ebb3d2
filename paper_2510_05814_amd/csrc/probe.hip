// Issue-rate probe for the roofline's compute peak: how many wave64 FP32 VALU instructions a
// SIMD retires per cycle in a loop of independent chains.  kind 0: fma with vector operands
// only; kind 1: fma reading a scalar register; kind 2: v_exp_f32.  Each thread
// runs 8 independent chains for `iters` iterations and stores their sum (so that nothing is
// optimised away).  Built like every kernel here (no packed FP32).
#include "tile_math.h"

namespace smoe {
namespace {

template <int KIND>
__global__ __launch_bounds__(256) void k_issue_probe(float* __restrict__ out, int iters, float a,
                                                     float b) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 0.25f + 0.01f * (float)((gid + k) & 7);
  // kind 0 keeps the multiplier and addend in vector registers; kind 1 leaves them to the
  // compiler, which reads them from scalar registers
  const float av = KIND == 1 ? a : in_vgpr(a);
  const float bv = KIND == 1 ? b : in_vgpr(b);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (KIND == 2) x[k] = __builtin_amdgcn_exp2f(-x[k]);
      else x[k] = __builtin_fmaf(x[k], av, bv);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[gid] = s;
}

}  // namespace

hipError_t launch_issue_probe(int kind, int iters, int workgroups, float* out, hipStream_t s) {
  if (kind == 0) k_issue_probe<0><<<workgroups, 256, 0, s>>>(out, iters, 0.999f, 0.001f);
  else if (kind == 1) k_issue_probe<1><<<workgroups, 256, 0, s>>>(out, iters, 0.999f, 0.001f);
  else k_issue_probe<2><<<workgroups, 256, 0, s>>>(out, iters, 0.999f, 0.001f);
  return hipGetLastError();
}

}  // namespace smoe
