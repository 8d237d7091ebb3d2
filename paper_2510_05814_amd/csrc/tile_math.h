// Per-block math of the rasterized SMoE on gfx950, shared by the standalone render and
// backward calls and the fused fit-step kernel.  Internal header.
//
// Lane layout: one wave per 16x16 block; lane l owns column l & 15 and the four rows
// (l >> 4) + 4i, i = 0..3.  The column-only terms of the exact truncation test (dx, z1,
// l21 z1, z1^2) are then computed once per kernel for the lane's four pixels, and a wave
// iteration i covers one 16x4 strip of the block.
#pragma once

#include "device_common.h"

namespace smoe {

constexpr int kWave = 64;

// Compile-time shape of a launch: channels, expert order, regression mode (RBF: the
// un-normalised sum of Eq. 1 instead of the gated SMoE of Eq. 2-4) and the reading of the
// truncation (which bound the render applies).
template <int C_, int ORDER_, bool RBF_, int TRUNC_>
struct Shape {
  static constexpr int C = C_, ORDER = ORDER_, TRUNC = TRUNC_;
  static constexpr bool RBF = RBF_;
};

// Calls f(Shape<...>{}) for the run-time (C, order, mode, reading); C is 1 or 3, order 0 or 1.
template <int C, int ORDER, class F>
inline void with_mode(const Segs& S, F&& f) {
  const bool rbf = S.mode == SMOE_MODE_RBF;
  if (S.trunc == SMOE_TRUNC_RENDER)
    rbf ? f(Shape<C, ORDER, true, SMOE_TRUNC_RENDER>{}) : f(Shape<C, ORDER, false, SMOE_TRUNC_RENDER>{});
  else
    rbf ? f(Shape<C, ORDER, true, SMOE_TRUNC_GRADIENT>{})
        : f(Shape<C, ORDER, false, SMOE_TRUNC_GRADIENT>{});
}
template <class F>
inline void with_shape(int C, int order, const Segs& S, F&& f) {
  if (C == 1 && order == 0) with_mode<1, 0>(S, f);
  else if (C == 1 && order == 1) with_mode<1, 1>(S, f);
  else if (C == 3 && order == 0) with_mode<3, 0>(S, f);
  else with_mode<3, 1>(S, f);
}
constexpr int kChunk = 64;                     // records staged in LDS per chunk
constexpr int kRows = kTilePixels / kWave;     // pixels per lane (4)

struct PixelCoords {
  int u;            // output column of the lane (within its raster; < 0 or >= W: outside)
  int v0;           // output row of the lane's first pixel (rows v0 + 4i)
  float x;          // sampling coordinates
  float y[kRows];
};

// Whether output pixel (u, v) lies in the raster (the first and last blocks of a window may
// hang over its edges).
__device__ __forceinline__ bool in_raster(int u, int v, const SegGrid& g) {
  return (unsigned)u < (unsigned)g.W && (unsigned)v < (unsigned)g.H;
}

// `tile` is the block index inside the segment's raster.  The raster's blocks are aligned
// to multiples of 16 in the output coordinate o + u (SegGrid), so the block's first column
// is u = 16 (bx0 + tx) - ox.  A native block is 16 s output pixels and begins on such a
// multiple (binary32 sample coordinates included, over the whole accepted range of origins,
// sizes and scales), so all of a block's points lie in one native block and every kernel of
// its list is a member at every one of them: no per-point membership test.
__device__ __forceinline__ PixelCoords lane_pixels(const SegGrid& g, int tile) {
  PixelCoords p;
  const int lane = threadIdx.x & 63;
  const int tx = tile % g.ntx, ty = tile / g.ntx;
  p.u = kTile * (g.bx0 + tx) - g.ox + (lane & 15);
  p.v0 = kTile * (g.by0 + ty) - g.oy + (lane >> 4);
  p.x = sample_coord(p.u, g.ox, g.inv_s);
#pragma unroll
  for (int i = 0; i < kRows; ++i) p.y[i] = sample_coord(p.v0 + 4 * i, g.oy, g.inv_s);
  return p;
}

// Stages the records of list entries [base, base + n) (n <= kChunk) into LDS.  An entry
// holds the kernel id shifted left by `shift` (the fit step's packed bucket entries; 0
// elsewhere).
template <int RS>
__device__ __forceinline__ void stage_records(float4* __restrict__ srec,
                                              const float* __restrict__ records,
                                              const uint32_t* __restrict__ vals, int base, int n,
                                              int shift) {
  constexpr int Q = RS / 4;
  __syncthreads();
  for (int i = threadIdx.x & 63; i < n * Q; i += kWave) {
    const int k = i / Q, c = i - k * Q;
    srec[i] = reinterpret_cast<const float4*>(records + (size_t)(vals[base + k] >> shift) * RS)[c];
  }
  __syncthreads();
}

// The same with the entries in LDS: ent[k] is entry base + k, copied there from vals first
// unless `ready` (the caller's sort left the list there).
template <int RS>
__device__ __forceinline__ void stage_records_lds(float4* __restrict__ srec,
                                                  const float* __restrict__ records,
                                                  const uint32_t* __restrict__ vals, int base,
                                                  int n, int shift, uint32_t* __restrict__ ent,
                                                  bool ready) {
  constexpr int Q = RS / 4;
  __syncthreads();
  if (!ready) {
    const int lane = threadIdx.x & 63;
    if (lane < n) ent[lane] = vals[base + lane];
    __syncthreads();
  }
  for (int i = threadIdx.x & 63; i < n * Q; i += kWave) {
    const int k = i / Q, c = i - k * Q;
    srec[i] = reinterpret_cast<const float4*>(records + (size_t)(ent[k] >> shift) * RS)[c];
  }
  __syncthreads();
}

// One list entry of the forward: adds its terms to D = sum pi K and N_c = sum pi K m_c of
// the lane's four pixels that the render's rule keeps.  TRUNC == SMOE_TRUNC_RENDER: the
// ellipse q <= r^2.  TRUNC == SMOE_TRUNC_GRADIENT (the block lists decide the render): every
// term binary32 holds, i.e. whose exponent a = rho log2(e) - q log2(e)/2 is >= -125.  Returns
// whether any of the lane's pixels passed the ellipse test q <= r2.  r: the entry's render
// record; cut_scale, cut_offset: the render's bound in the compare-free form of Segs.
//
// Neither bound is a per-row compare: a VALU instruction that writes or reads a scalar
// register (a compare's lane mask, a select on it) issues at about 60 % of the rate of one
// on vector registers alone.  The ellipse test compares the minimum of the four rows' q
// once; the render's bound goes through the exponent: with the ellipse, max(q, u) with
// u = fma(q, cut_scale, cut_offset) is q inside the bound and gives a term beyond it an
// exponent of about -2^36; with the representable range, min(a, fma(a, 2^60, 125 * 2^60)) is
// a for a >= -125 and below -2^43 otherwise.  Either way exp2 of an excluded term is exactly
// zero and every kept term carries the same bits as with a compare-and-select.
template <int C, int ORDER, int TRUNC>
__device__ __forceinline__ bool forward_entry(const PixelCoords& px, float r2, float cut_scale,
                                              float cut_offset, const float* r, float (&D)[kRows],
                                              float (&N)[kRows][C]) {
  // Truncation test: the binary32 sequence of the ABI contract (no contraction).
  const float dx = px.x - r[0];
  const float z1 = dx * r[2];
  const float tt = r[3] * z1;
  const float zz1 = z1 * z1;
  // a_c + wx_c dx: the expert's value along the lane's column
  float mx[C];
#pragma unroll
  for (int c = 0; c < C; ++c)
    mx[c] = ORDER == 1 ? __builtin_fmaf(r[kRecExpert + C + c], dx, r[kRecExpert + c])
                       : r[kRecExpert + c];
  float q[kRows], dy[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    dy[i] = px.y[i] - r[1];
    const float w = dy[i] - tt;
    const float z2 = w * r[4];
    q[i] = zz1 + z2 * z2;
  }
  // pi K = exp(rho - q/2) = exp2(rho log2 e - q log2 e / 2), with the render's bound applied
  // in its compare-free form -- which is the identity, bit for bit, unless some pixel of the
  // block lies beyond the bound (q > r^2 with the ellipse in the render; an exponent below
  // -125 otherwise), so the wave applies it only then.
  float a[kRows];
  if (TRUNC == SMOE_TRUNC_RENDER) {
    const float qmax = __builtin_fmaxf(__builtin_fmaxf(q[0], q[1]), __builtin_fmaxf(q[2], q[3]));
    if (__any(!(qmax <= r2))) {
#pragma unroll
      for (int i = 0; i < kRows; ++i)
        q[i] = __builtin_fmaxf(q[i], __builtin_fmaf(q[i], cut_scale, cut_offset));
    }
#pragma unroll
    for (int i = 0; i < kRows; ++i) a[i] = __builtin_fmaf(q[i], -0.5f * kLog2e, r[5]);
  } else {
#pragma unroll
    for (int i = 0; i < kRows; ++i) a[i] = __builtin_fmaf(q[i], -0.5f * kLog2e, r[5]);
    const float amin = __builtin_fminf(__builtin_fminf(a[0], a[1]), __builtin_fminf(a[2], a[3]));
    if (__any(!(amin >= -125.0f))) {
#pragma unroll
      for (int i = 0; i < kRows; ++i)
        a[i] = __builtin_fminf(a[i], __builtin_fmaf(a[i], cut_scale, cut_offset));
    }
  }
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const float e = __builtin_amdgcn_exp2f(a[i]);
    D[i] += e;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float m = mx[c];
      if (ORDER == 1) m = __builtin_fmaf(r[kRecExpert + 2 * C + c], dy[i], m);
      N[i][c] = __builtin_fmaf(e, m, N[i][c]);
    }
  }
  static_assert(kRows == 4, "the ellipse test takes the minimum of four rows");
  // q >= +0 (a sum of squares, or the bound's larger stand-in), so the order of the floats is
  // the order of their bit patterns as integers: no NaN handling in the minimum
  const int qmin = min(min(__float_as_int(q[0]), __float_as_int(q[1])),
                       min(__float_as_int(q[2]), __float_as_int(q[3])));
  return __int_as_float(qmin) <= r2;
}

// A copy of x that the compiler must keep in a vector register: loop-invariant operands of
// the forward's per-row arithmetic are read from VGPRs rather than SGPRs (see forward_entry).
__device__ __forceinline__ float in_vgpr(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int C>
__device__ __forceinline__ void zero_sums(float (&D)[kRows], float (&N)[kRows][C]) {
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    D[i] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) N[i][c] = 0.0f;
  }
}

// Forward accumulation over a block's list [rg.x, rg.y) in list order (forward_entry per
// entry, records staged through LDS in chunks).
// live: bit k set if any pixel of the block passed the ellipse test q <= r2 for entry k of
// the last staged chunk (the only chunk for lists of up to kChunk entries).
// shift: list entries hold the kernel id << shift.  ent: null, or LDS room for one chunk of
// entries, which the staging then reads from there (a single-chunk list already holds them,
// sorted; longer lists copy each chunk's entries in).
template <int C, int ORDER, int TRUNC>
__device__ __forceinline__ void forward_accumulate(const PixelCoords& px, float r2,
                                                   float cut_scale, float cut_offset,
                                                   const float* __restrict__ records,
                                                   const uint32_t* __restrict__ vals, int shift,
                                                   int2 rg, float4* srec, float (&D)[kRows],
                                                   float (&N)[kRows][C], uint64_t& live,
                                                   uint32_t* ent = nullptr) {
  constexpr int RS = record_stride(C, ORDER);
  constexpr int Q = RS / 4;
  zero_sums<C>(D, N);
  cut_scale = in_vgpr(cut_scale);
  cut_offset = in_vgpr(cut_offset);
  for (int base = rg.x; base < rg.y; base += kChunk) {
    const int n = min(kChunk, rg.y - base);
    if (ent) stage_records_lds<RS>(srec, records, vals, base, n, shift, ent, rg.y - rg.x <= kChunk);
    else stage_records<RS>(srec, records, vals, base, n, shift);
    live = 0;
    for (int k = 0; k < n; ++k) {
      const float* r = reinterpret_cast<const float*>(&srec[k * Q]);
      if (__any(forward_entry<C, ORDER, TRUNC>(px, r2, cut_scale, cut_offset, r, D, N)))
        live |= 1ull << k;
    }
  }
}

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

// Transposed reduction inside each 16-lane row: on return lane l holds the sum over the
// row's 16 lanes of v[l & 15].  Stages pair lane l with l ^ 8 (row_ror:8), with 7 - l in its
// group of 8 (row_half_mirror), then l ^ 2 and l ^ 1 (quad_perm); at each stage a lane keeps
// the half of its values selected by that bit of its index and adds the partner's copy.
// Every lane of the row must be active.
__device__ __forceinline__ float row_reduce16_transposed(float (&v)[16]) {
  const int lane = threadIdx.x & 63;
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0,
             b0 = (lane & 1) != 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float keep = b3 ? v[i + 8] : v[i], send = b3 ? v[i] : v[i + 8];
    v[i] = keep + dpp<0x128>(send);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = b2 ? v[i + 4] : v[i], send = b2 ? v[i] : v[i + 4];
    v[i] = keep + dpp<0x141>(send);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b1 ? v[i + 2] : v[i], send = b1 ? v[i] : v[i + 2];
    v[i] = keep + dpp<0x4E>(send);
  }
  const float keep = b0 ? v[1] : v[0], send = b0 ? v[0] : v[1];
  return keep + dpp<0xB1>(send);
}

// Adds partial row p (NP values of a row of partial_stride(NP) floats) to v.
template <int NP>
__device__ __forceinline__ void add_partial_row(float (&v)[16], const float* __restrict__ pair_grads,
                                                int p) {
  constexpr int PS = partial_stride(NP);
  const float4* row = reinterpret_cast<const float4*>(pair_grads + (size_t)p * PS);
#pragma unroll
  for (int q4 = 0; q4 < PS / 4; ++q4) {
    const float4 x = row[q4];
    if (4 * q4 + 0 < NP) v[4 * q4 + 0] += x.x;
    if (4 * q4 + 1 < NP) v[4 * q4 + 1] += x.y;
    if (4 * q4 + 2 < NP) v[4 * q4 + 2] += x.z;
    if (4 * q4 + 3 < NP) v[4 * q4 + 3] += x.w;
  }
}

// The position of kernel j in block t's sorted list (a binary search; entries hold the
// kernel id << shift), or -1 if the list does not hold j.
__device__ __forceinline__ int list_position(int j, int t, const int2* __restrict__ ranges,
                                             const uint32_t* __restrict__ vals, int shift) {
  const int2 rg = ranges[t];
  if (rg.y <= rg.x) return -1;
  return find_in_list(vals, rg.x, rg.y, (uint32_t)j, shift);
}

// Gradient of kernel row j: the sum of its per-block partial rows over its block rectangle.
// A group of 16 lanes (one 16-lane row of the wave) serves one kernel: lane b adds the partial
// rows of blocks b, b + 16, ... of the rectangle (row-major); the row reduction then leaves
// parameter i's gradient in lane i.  The summation order is fixed, so the result is
// reproducible.  The standalone backward's partial row of a (block, kernel) pair is at the
// pair's list position, found by a search.  All 16 lanes must call it (live = false: the
// kernel contributes nothing).
template <int NP>
__device__ __forceinline__ float gather_param(int j, bool live, const SegGrid& sg,
                                              const int4* __restrict__ rects,
                                              const int2* __restrict__ ranges,
                                              const uint32_t* __restrict__ vals,
                                              const float* __restrict__ pair_grads) {
  static_assert(NP <= 16, "16 lanes per kernel");
  float v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = 0.0f;
  if (live) {
    const int4 rc = rects[j];
    const int n = rect_count(rc);
    const int w = rc.z - rc.x + 1;
    for (int b = threadIdx.x & 15; b < n; b += 16) {
      const int dy = b / w;
      const int p = list_position(j, sg.tile_offset + (rc.y + dy) * sg.ntx + rc.x + (b - dy * w),
                                  ranges, vals, 0);
      if (p >= 0) add_partial_row<NP>(v, pair_grads, p);
    }
  }
  return row_reduce16_transposed(v);
}

// The fit step's gather, in the same order, with the kernel's rectangle rc already loaded by
// the caller.  The partial row of the kernel's block b is at row kSlots j + b for b < kSlots
// (contiguous per kernel); beyond, at row kSlots K + the bucket slot that the entry's low bits
// hold, found by a search of the block's sorted list.
template <int NP>
__device__ __forceinline__ float gather_param_fit(int j, bool live, const SegGrid& sg, int4 rc,
                                                  int K, const int2* __restrict__ ranges,
                                                  const uint32_t* __restrict__ vals,
                                                  const float* __restrict__ pair_grads,
                                                  int shift) {
  static_assert(NP <= 16, "16 lanes per kernel");
  float v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = 0.0f;
  if (live) {
    const int n = rect_count(rc);
    const int w = rc.z - rc.x + 1;
    for (int b = threadIdx.x & 15; b < n; b += 16) {
      int p = j * kSlots + b;
      if (b >= kSlots) {
        const int dy = b / w;
        const int t = sg.tile_offset + (rc.y + dy) * sg.ntx + rc.x + (b - dy * w);
        const int pos = list_position(j, t, ranges, vals, shift);
        if (pos < 0) continue;
        const int low = (int)(vals[pos] & ((1u << shift) - 1u));
        p = K * kSlots + ranges[t].x + (low - kSlots);
      }
      add_partial_row<NP>(v, pair_grads, p);
    }
  }
  return row_reduce16_transposed(v);
}

// A kernel's gradient from the sums of its partial rows (lane i of the kernel's 16-lane group
// holds the sum of field i; every lane of the group must call it).  Fields 0 and 1 of a
// partial row leave out the expert terms of the centre's gradient, which factor through the
// kernel's slopes and are applied here once per kernel:
//   dL/dmu_x = field 0 - sum_c wx_c dL/da_c,  dL/dmu_y = field 1 - sum_c wy_c dL/da_c.
// slopes: a per-lane value whose lane SLOPES + C + c holds wx_c and lane SLOPES + 2C + c
// holds wy_c (the render record's fields, or the kernel's raw row: the same numbers).
template <int C, int ORDER, int SLOPES>
__device__ __forceinline__ float finish_gradient(float s, bool live, float slopes) {
  if (ORDER == 0) return s;
  const int i = threadIdx.x & 15;
  float ex = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float da = __shfl(s, 6 + c, 16);
    const float slope = __shfl(slopes, SLOPES + ((i == 0) ? 1 : 2) * C + c, 16);
    ex = __builtin_fmaf(da, slope, ex);
  }
  return live && i < 2 ? s - ex : s;
}

// Adjoint seed of one pixel: dL/dy (g), 1/D, sum_c g_c y_c; `valid` false where D = 0 or the
// pixel lies outside the raster (no gradient flows there).  With the seed 1/D -> 1 and
// sum_c g_c y_c -> 0 the same backward is the adjoint of the un-normalised sum of Eq. (1):
// then w = pi K is dy_c/dm_c and G = sum_c g_c m_c is dL/d(pi K).
template <int C>
struct PixelSeed {
  float g[kRows][C];
  float invD[kRows];
  float gy[kRows];
  bool valid[kRows];
};

// Backward over a block's list [rg.x, rg.y): for every kernel the wave forms, per pixel, the
// adjoints of its 6 + 3C raw parameters (recomputing pi K from the record, w = pi K / D),
// sums them over the block's 256 pixels with the transposed reduction, and writes the
// per-(block, kernel) partial row pair_grads[list position].  `staged`: the records of a
// single-chunk list are already in srec and `live` holds the forward's per-entry hits (the
// fused fit kernel rendered from them): an entry no pixel passed gets a zero row without
// repeating its tests -- the row it would reduce to, bit for bit.
//   G = sum_c g_c (m_c - y_c),  H = w G                       (dL/drho)
//   dL/da_c = g_c w,  dL/dwx_c = g_c w dx,  dL/dwy_c = g_c w dy
//   bz2 = -H z2,  bz1 = -H z1 - bz2 l21/l22                  (through q = z1^2 + z2^2)
//   dL/dmu_x = -(bz1/l11 + sum_c g_c w wx_c),  dL/dmu_y = -(bz2/l22 + sum_c g_c w wy_c)
//   dL/ds1 = -bz1 z1,  dL/dl21 = -bz2 z1/l22,  dL/ds2 = -bz2 z2
// Fields 0 and 1 of the partial row leave out the sum_c g_c w wx_c and sum_c g_c w wy_c
// terms: the gather applies them per kernel from dL/da_c (finish_gradient).
// The terms that factor through a lane's column (dx, z1) or through the kernel (1/l11,
// 1/l22) are applied once per lane to the lane's sums instead of once per pixel; so is the
// l21/l22 term of bz1 (sum bz1 = -(z1 sum H + (l21/l22) sum bz2) over a lane's
// pixels), and the seeds g and sum_c g_c y_c are taken already divided by D, so that pi K
// itself stands in for w.
// packed (the fit step): list entries hold kernel id << shift | low, and the partial row of
// the entry goes to row kSlots j + low for low < kSlots (the block's index in the kernel's
// rectangle: kernel-major rows), else to row kSlots K + rg.x + low - kSlots (its bucket
// slot), where the fit step's gather reads it; otherwise to the entry's list position.
template <int C, int ORDER>
__device__ __forceinline__ void backward_accumulate(const PixelCoords& px, float r2,
                                                    const float* __restrict__ records,
                                                    const uint32_t* __restrict__ vals, int shift,
                                                    bool packed, int2 rg, float4* srec,
                                                    bool staged, uint64_t live,
                                                    const PixelSeed<C>& sd,
                                                    float* __restrict__ pair_grads,
                                                    int K = 0) {
  constexpr int RS = record_stride(C, ORDER);
  constexpr int Q = RS / 4;
  constexpr int NP = num_params(C, ORDER);
  constexpr int PS = partial_stride(NP);
  static_assert(PS <= 16, "16 accumulators per kernel");
  const int lane = threadIdx.x & 63;
  // the seeds divided by D: g_c / D and sum_c g_c y_c / D
  float gs[kRows][C], gys[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    gys[i] = sd.gy[i] * sd.invD[i];
#pragma unroll
    for (int c = 0; c < C; ++c) gs[i][c] = sd.g[i][c] * sd.invD[i];
  }
  for (int base = rg.x; base < rg.y; base += kChunk) {
    const int n = min(kChunk, rg.y - base);
    const bool reuse = staged && rg.y - rg.x <= kChunk;
    if (!reuse) stage_records<RS>(srec, records, vals, base, n, shift);
    const uint32_t slot_mask = (1u << shift) - 1u;
    // the row of entry k's partial: the one its low bits name (packed) or its list position
    auto out_row = [&](int k) -> size_t {
      if (!packed) return (size_t)(base + k);
      const uint32_t e = __builtin_amdgcn_readfirstlane(vals[base + k]);
      const uint32_t low = e & slot_mask;
      return low < (uint32_t)kSlots ? (size_t)(e >> shift) * kSlots + low
                                    : (size_t)K * kSlots + (size_t)rg.x + (low - kSlots);
    };
    for (int k = 0; k < n; ++k) {
      if (reuse && !((live >> k) & 1ull)) {
        // no pixel of the block passed the forward's test: the partial row is zero
        const int idx = lane >> 2;
        if ((lane & 3) == 0 && idx < PS) pair_grads[out_row(k) * PS + idx] = 0.0f;
        continue;
      }
      const float* r = reinterpret_cast<const float*>(&srec[k * Q]);
      const float dx = px.x - r[0];
      const float z1 = dx * r[2];
      const float tt = r[3] * z1;
      const float zz1 = z1 * z1;
      // a_c + wx_c dx: the expert's value along the lane's column
      float mx[C];
#pragma unroll
      for (int c = 0; c < C; ++c)
        mx[c] = ORDER == 1 ? __builtin_fmaf(r[kRecExpert + C + c], dx, r[kRecExpert + c])
                           : r[kRecExpert + c];
      // Per lane, over its four pixels: the sums that do not factor through the lane's
      // column -- A_c = sum g_c w, Y_c = sum g_c w dy, V = sum H (dy - t), S2 = sum H z2^2,
      // R = sum H.  dx and z1 are the same for the lane's pixels, so sum g_c w dx = dx A_c,
      // sum bz2 = -V / l22 (z2 = (dy - t) / l22), sum bz1 = -(z1 R + (l21/l22) sum bz2),
      // sum bz1 z1 = z1 sum bz1 and sum g_c w wx_c = wx_c A_c.  With the seeds divided by D,
      // w = pi K / D is e = pi K.
      float A[C], Y[C];
#pragma unroll
      for (int c = 0; c < C; ++c) A[c] = Y[c] = 0.0f;
      float V = 0.0f, S2 = 0.0f, R = 0.0f;
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        const float dy = px.y[i] - r[1];
        const float w_ = dy - tt;
        const float z2 = w_ * r[4];
        const float z2sq = z2 * z2;
        const float q = zz1 + z2sq;
        // the first row runs unmasked with pi K zeroed where it does not take part, so that
        // it can start the sums without zero-filled accumulators in front of it
        const bool ok = sd.valid[i] && q <= r2;
        if (i == 0 || ok) {
          float e = __builtin_amdgcn_exp2f(__builtin_fmaf(q, -0.5f * kLog2e, r[5]));
          if (i == 0) e = ok ? e : 0.0f;
          const float ed = e * dy;
          float Gs = -gys[i];  // G / D
#pragma unroll
          for (int c = 0; c < C; ++c) {
            float m = mx[c];
            if (ORDER == 1) m = __builtin_fmaf(r[kRecExpert + 2 * C + c], dy, m);
            Gs = __builtin_fmaf(gs[i][c], m, Gs);
            // the first row's terms start the sums: no additions of zero
            A[c] = i == 0 ? gs[i][c] * e : __builtin_fmaf(gs[i][c], e, A[c]);
            if (ORDER == 1) Y[c] = i == 0 ? gs[i][c] * ed : __builtin_fmaf(gs[i][c], ed, Y[c]);
          }
          const float Hh = e * Gs;  // H = w G
          V = i == 0 ? Hh * w_ : __builtin_fmaf(Hh, w_, V);
          S2 = i == 0 ? Hh * z2sq : __builtin_fmaf(Hh, z2sq, S2);
          R = i == 0 ? Hh : R + Hh;
        }
      }
      const float B2 = -V * r[4];
      const float B1 = -__builtin_fmaf(r[6], B2, z1 * R);
      // fields 0 and 1 leave the expert terms of the centre's gradient to finish_gradient
      float acc[16];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc[6 + c] = A[c];
        if (ORDER == 1) {
          acc[6 + C + c] = A[c] * dx;
          acc[6 + 2 * C + c] = Y[c];
        }
      }
      acc[0] = -B1 * r[2];
      acc[1] = -B2 * r[4];
      acc[2] = -B1 * z1;
      acc[3] = -B2 * z1 * r[4];
      acc[4] = S2;
      acc[5] = R;
#pragma unroll
      for (int i = 6 + C * (1 + 2 * ORDER); i < 16; ++i) acc[i] = 0.0f;
      const float tot = wave_reduce16_transposed(acc);
      const int idx = lane >> 2;
      if ((lane & 3) == 0 && idx < PS) pair_grads[out_row(k) * PS + idx] = tot;
    }
  }
}

}  // namespace smoe
