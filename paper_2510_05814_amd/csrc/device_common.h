// Device building blocks shared by the standalone binning calls and the fused fit step:
// the kernel box (Sec. IV-B), the render record, the per-block ordering of a bucket and the
// block scan that turns per-block counts into list ranges (Sec. IV-C).  Internal header.
#pragma once

#include "smoe_internal.h"

namespace smoe {

constexpr int kStepShadow = 4;  // status word: completed steps, copied by the step's first kernel
constexpr int kStepFlags = 5;   // status words 5, 6: the fit step's overflow flag by step parity
constexpr int kNonfinite = 7;   // status word: a kernel row with a NaN or infinite parameter was
                                // seen (cleared by each binning's first kernel and at the start
                                // of a fit; sticky over a fit's steps)
constexpr int kNonfiniteOut = 3;  // status word: the binning's copy of kNonfinite

// Native 16x16 block index of a native coordinate, floor(x / 16) (x * 2^-4 is exact).
__device__ __forceinline__ float native_block(float x) { return floorf(x * 0.0625f); }

// Output-block range [t0, t1] of one axis of a raster (n points sampled at
// ((o + u) + 0.5) * inv_s; blocks aligned to multiples of 16 in o + u) holding a point whose
// native block lies in [b0, b1], and the
// native range clamped to the blocks the raster's points reach.  The native block index does
// not decrease along the axis, so the points form one run [u0, u1]: at scale 1 the block of
// point u is (o + u) >> 4 exactly; otherwise both ends are found by binary search over the
// exact binary32 sample coordinates.  False when no point is in [b0, b1] (or NaN).
__device__ __forceinline__ bool output_axis(float b0, float b1, int n, int o, int scale,
                                            float inv_s, int& t0, int& t1, int& nb0, int& nb1) {
  const float first = native_block(sample_coord(0, o, inv_s));
  const float last = native_block(sample_coord(n - 1, o, inv_s));
  if (!(b1 >= first) || !(b0 <= last)) return false;
  nb0 = (int)fmaxf(b0, first);
  nb1 = (int)fminf(b1, last);
  int u0, u1;
  if (scale == 1) {
    u0 = max(0, 16 * nb0 - o);
    u1 = min(n - 1, 16 * nb1 + 15 - o);
  } else {
    // first point with native block >= nb0, and first point with native block > nb1
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (native_block(sample_coord(mid, o, inv_s)) >= (float)nb0) hi = mid;
      else lo = mid + 1;
    }
    u0 = lo;
    lo = 0;
    hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (native_block(sample_coord(mid, o, inv_s)) > (float)nb1) hi = mid;
      else lo = mid + 1;
    }
    u1 = lo - 1;
  }
  // blocks of the grid aligned to multiples of 16 in o + u, numbered from the raster's first
  t0 = first_block(o + u0) - first_block(o);
  t1 = first_block(o + u1) - first_block(o);
  return true;
}

// A kernel's blocks on one raster: `tile` = its output-block rectangle (tx0, ty0, tx1, ty1)
// and `native` = its native 16x16 blocks (bx0, by0, bx1, by1) clamped to those the raster's
// points reach; both (0, 0, -1, -1) when empty.
struct KernelRects {
  int4 tile, native;
};

// The blocks of one kernel: the native blocks its square box of half-side
// R = r sqrt(lambda_max(L L^T)) around mu covers -- with the block lists deciding the render
// (SMOE_TRUNC_GRADIENT) those holding a native pixel centre inside the box, with the ellipse
// deciding (SMOE_TRUNC_RENDER) those the box overlaps, so that every point inside the ellipse
// is a member at any scale -- or those of its tight axis-aligned box of the
// ellipse's x and y extents (widened by a rounding margin, capped at R) -- as the exact
// binary32 sequences of the ABI contract; the raster's output blocks are those holding a
// sample point in them.
__device__ __forceinline__ KernelRects kernel_rects(float mux, float muy, float l11, float l21,
                                                    float l22, const SegGrid& g, float r, int box,
                                                    int trunc) {
  const float sxx = l11 * l11;
  const float sxy = l11 * l21;
  const float syy = l21 * l21 + l22 * l22;
  const float h = 0.5f * (sxx + syy);
  const float d = 0.5f * (sxx - syy);
  const float lam = h + sqrtf(d * d + sxy * sxy);
  const float R = r * sqrtf(lam);
  float Rx = R, Ry = R;
  if (box == SMOE_BOX_TIGHT) {
    const float m = (fabsf(mux) + fabsf(muy) + R) * 0x1p-18f;
    Rx = fminf(R, r * fabsf(l11) * 1.0009765625f + m);
    Ry = fminf(R, r * sqrtf(syy) * 1.0009765625f + m);
  }
  float bx0f, bx1f, by0f, by1f;
  if (trunc == SMOE_TRUNC_GRADIENT) {
    // the blocks of the native pixel centres c + 0.5 inside the box: c from ceil(lo - 0.5)
    // to floor(hi - 0.5) (empty if none)
    const float cx0 = ceilf((mux - Rx) - 0.5f), cx1 = floorf((mux + Rx) - 0.5f);
    const float cy0 = ceilf((muy - Ry) - 0.5f), cy1 = floorf((muy + Ry) - 0.5f);
    bx0f = cx0 <= cx1 ? native_block(cx0) : 1.0f;
    bx1f = cx0 <= cx1 ? native_block(cx1) : 0.0f;
    by0f = cy0 <= cy1 ? native_block(cy0) : 1.0f;
    by1f = cy0 <= cy1 ? native_block(cy1) : 0.0f;
  } else {
    // the blocks the box overlaps: floor(lo/16) .. ceil(hi/16) - 1
    bx0f = native_block(mux - Rx);
    bx1f = ceilf((mux + Rx) * 0.0625f) - 1.0f;
    by0f = native_block(muy - Ry);
    by1f = ceilf((muy + Ry) * 0.0625f) - 1.0f;
  }
  KernelRects k;
  k.tile = make_int4(0, 0, -1, -1);
  k.native = make_int4(0, 0, -1, -1);
  if (!(bx0f <= bx1f) || !(by0f <= by1f)) return k;
  int tx0, tx1, ty0, ty1, bx0, bx1, by0, by1;
  if (output_axis(bx0f, bx1f, g.W, g.ox, g.scale, g.inv_s, tx0, tx1, bx0, bx1) &&
      output_axis(by0f, by1f, g.H, g.oy, g.scale, g.inv_s, ty0, ty1, by0, by1)) {
    k.tile = make_int4(tx0, ty0, tx1, ty1);
    k.native = make_int4(bx0, by0, bx1, by1);
  }
  return k;
}

// n / d from r = v_rcp_f32(d) (within 1 ulp of 1/d) and one Newton-Raphson correction of
// the quotient: q = n r, q + r (n - d q).  Within an ulp of the correctly rounded quotient
// (equal to it in all but about 5 of 10^7 random cases), and exactly 1 when n == d, so the
// gates still sum to one bit for bit; a few instructions instead of the scaled IEEE
// division sequence.
__device__ __forceinline__ float div_refined(float n, float d, float r) {
  const float q = n * r;
  return __builtin_fmaf(__builtin_fmaf(-d, q, n), r, q);
}

__device__ __forceinline__ int rect_count(int4 rc) {
  return rc.z < rc.x ? 0 : (rc.z - rc.x + 1) * (rc.w - rc.y + 1);
}

// One increment per covered block (global block ids): the histogram of the block-id digit.
__device__ __forceinline__ void count_blocks(int4 rc, const SegGrid& g,
                                             int32_t* __restrict__ tile_counts, int first = 0,
                                             int stride = 1) {
  const int n = rect_count(rc), w = rc.z - rc.x + 1;
  for (int q = first; q < n; q += stride)
    atomicAdd(&tile_counts[g.tile_offset + (rc.y + q / w) * g.ntx + rc.x + q % w], 1);
}

// Float4 number `quad` of the render record of a kernel row from its materialized parameter
// row p (layout in smoe_internal.h; the record is 16-byte aligned): field f holds, beyond the
// seven geometry fields, expert float f - 7 = p[f - 1], and zero padding after the experts.
// (l11, l21, l22): the Cholesky factor the record is built for (the row's own, or divided by
// a sharpening factor).
__device__ __forceinline__ void write_record_quad(float* __restrict__ rec,
                                                  const float* __restrict__ p, int ne, int quad,
                                                  float l11, float l21, float l22) {
  float4* r4 = reinterpret_cast<float4*>(rec);
  if (quad == 0) {
    r4[0] = make_float4(p[0], p[1], 1.0f / l11, l21);
  } else if (quad == 1) {
    const float i22 = 1.0f / l22;
    r4[1] = make_float4(i22, p[5] * kLog2e, l21 * i22, ne > 0 ? p[6] : 0.0f);
  } else {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int f = 4 * quad + k;
      v[k] = f < kRecExpert + ne ? p[f - 1] : 0.0f;
    }
    r4[quad] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Exclusive scan of per-block counts into [begin, end) ranges by one workgroup of NT
// threads (NT = 1024), with P, the overflow flag and the longest list into status, and
// the counters reset to zero (they serve as the scatter cursors).  Each pass covers a
// chunk of 16*NT blocks: every thread holds 16 consecutive counts in registers (four
// int4 loads, contiguous across the wave), thread totals are scanned with wave shuffles
// and one exchange of wave totals, and the begins go through LDS so that ranges and
// resets are stored with consecutive threads on consecutive blocks.  Rasters of at most
// one chunk (16384 blocks, 2048^2 pixels) take a single pass; larger ones first sum all
// counts (P must be known before any range is written, so that an overflow can write
// every range empty).  s_begin: 16*NT ints; s_tot: NT/64 long longs.
template <int NT>
__device__ void block_scan_ranges(int T, int32_t* __restrict__ tile_counts,
                                  int2* __restrict__ ranges, int capacity,
                                  int32_t* __restrict__ status, int* s_begin, long long* s_tot) {
  constexpr int ITEMS = 16;
  constexpr int CHUNK = NT * ITEMS;
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int s_max[NW];
  long long P = -1;  // unknown until summed
  int longest = 0;
  if (T > CHUNK) {
    long long sum = 0;
    int mx = 0;
    for (int t0 = tid * 4; t0 < T; t0 += NT * 4) {
      if (t0 + 4 <= T) {
        const int4 v = *reinterpret_cast<const int4*>(tile_counts + t0);
        sum += (long long)v.x + v.y + v.z + v.w;
        mx = max(mx, max(max(v.x, v.y), max(v.z, v.w)));
      } else {
        for (int q = t0; q < T; ++q) {
          sum += tile_counts[q];
          mx = max(mx, tile_counts[q]);
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      sum += __shfl_xor(sum, off);
      mx = max(mx, __shfl_xor(mx, off));
    }
    if (lane == 0) {
      s_tot[wave] = sum;
      s_max[wave] = mx;
    }
    __syncthreads();
    P = 0;
    for (int w = 0; w < NW; ++w) {
      P += s_tot[w];
      longest = max(longest, s_max[w]);
    }
    __syncthreads();
  }
  long long carry = 0;
  bool over = P > (long long)capacity;
  for (int base = 0; base < T; base += CHUNK) {
    const int b = base + tid * ITEMS;
    int c[ITEMS];
    if (b + ITEMS <= T) {
      const int4* p4 = reinterpret_cast<const int4*>(tile_counts + b);
#pragma unroll
      for (int q = 0; q < ITEMS / 4; ++q) {
        const int4 v = p4[q];
        c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) c[q] = (b + q < T) ? tile_counts[b + q] : 0;
    }
    long long local = 0;
    int mx = 0;
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      local += c[q];
      mx = max(mx, c[q]);
    }
    long long incl = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
    if (lane == 63) s_tot[wave] = incl;
    if (lane == 0) s_max[wave] = mx;
    __syncthreads();
    long long wbase = 0, ctot = 0;
    for (int w = 0; w < NW; ++w) {
      const long long t = s_tot[w];
      if (w < wave) wbase += t;
      ctot += t;
    }
    if (T <= CHUNK) {  // single pass: the chunk total is P
      P = ctot;
      over = P > (long long)capacity;
      for (int w = 0; w < NW; ++w) longest = max(longest, s_max[w]);
    }
    // Begins relative to the chunk; they fit in int32 whenever ranges are written (P is
    // then at most the int32 capacity).
    long long run = wbase + incl - local;
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      s_begin[tid * ITEMS + q] = (int)run;
      run += c[q];
    }
    __syncthreads();
    const int n = min(CHUNK, T - base);
    for (int i = tid; i < n; i += NT) {
      const int bg = (int)carry + s_begin[i];
      const int en = (i + 1 < n) ? (int)carry + s_begin[i + 1] : (int)(carry + ctot);
      ranges[base + i] = over ? make_int2(0, 0) : make_int2(bg, en);
      tile_counts[base + i] = 0;
    }
    carry += ctot;
    __syncthreads();
  }
  if (tid == 0) {
    status[0] = (int)min(P, (long long)INT32_MAX);
    status[1] = over ? 1 : 0;
    status[2] = longest;
    status[kNonfiniteOut] = status[kNonfinite];
  }
}

// Sorts one bucket of n distinct kernel ids (seg[0, n)) ascending with the 64 lanes of one
// wave: bitonic sort in LDS for runs of up to `run` ids (lds holds `run` u32), then
// pairwise merges of sorted runs in global memory through alt[0, n) for longer buckets.
// Only wave-level barriers are used (the caller's workgroup is this one wave).
// Sorts a bucket of n <= 64 distinct entries seg[0, n) ascending with one wave: each lane
// takes one entry, counts the bucket's entries below it (its rank) from broadcast reads of
// the whole bucket in LDS, and stores it at its rank, into `out` (LDS, kept for the caller)
// (if not null) and back into seg.  scratch: 64 u32 of LDS.
__device__ __forceinline__ void rank_sort64(uint32_t* __restrict__ seg, int n,
                                            uint32_t* __restrict__ scratch,
                                            uint32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const uint32_t e = lane < n ? seg[lane] : 0xFFFFFFFFu;
  scratch[lane] = e;  // padding above n: no entry is greater
  __syncthreads();
  int rank = 0;
  const uint4* s4 = reinterpret_cast<const uint4*>(scratch);
  for (int j = 0; j < (n + 3) >> 2; ++j) {
    const uint4 q = s4[j];
    rank += (q.x < e ? 1 : 0) + (q.y < e ? 1 : 0) + (q.z < e ? 1 : 0) + (q.w < e ? 1 : 0);
  }
  if (lane < n) {
    if (out) out[rank] = e;
    seg[rank] = e;
  }
  __threadfence_block();
  __syncthreads();
}

__device__ __forceinline__ void sort_bucket(uint32_t* __restrict__ seg, uint32_t* __restrict__ alt,
                                            int n, uint32_t* lds, int run) {
  const int lane = threadIdx.x & 63;
  if (n <= 1) return;
  for (int c0 = 0; c0 < n; c0 += run) {
    const int m = min(run, n - c0);
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    for (int i = lane; i < p2; i += 64) lds[i] = (i < m) ? seg[c0 + i] : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int i = lane; i < p2; i += 64) {
          const int ixj = i ^ jj;
          if (ixj > i) {
            const uint32_t a = lds[i], c = lds[ixj];
            if ((a > c) == ((i & k) == 0)) {
              lds[i] = c;
              lds[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = lane; i < m; i += 64) seg[c0 + i] = lds[i];
    __threadfence_block();
    __syncthreads();
  }
  if (n <= run) return;
  // An element's output position is its index in its own run plus the number of smaller
  // elements in the partner run.
  uint32_t* src = seg;
  uint32_t* dst = alt;
  for (int width = run; width < n; width <<= 1) {
    for (int i = lane; i < n; i += 64) {
      const int r_i = i / width;
      const int pair_lo = (r_i & ~1) * width;
      const bool left = (r_i & 1) == 0;
      const int o_lo = left ? min(n, pair_lo + width) : pair_lo;
      const int o_hi = left ? min(n, pair_lo + 2 * width) : pair_lo + width;
      const uint32_t v = src[i];
      int lo = o_lo, hi = o_hi;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (src[mid] < v) lo = mid + 1;
        else hi = mid;
      }
      dst[pair_lo + (i - r_i * width) + (lo - o_lo)] = v;
    }
    __threadfence_block();
    __syncthreads();
    uint32_t* tmp = src;
    src = dst;
    dst = tmp;
  }
  if (src != seg) {
    for (int i = lane; i < n; i += 64) seg[i] = src[i];
    __threadfence_block();
    __syncthreads();
  }
}

// Arguments the fit step's Adam kernel needs to record the loss and advance the step.
struct StepScalarsArgs {
  int32_t* step;
  float* scalars;
  float* loss_out;
  float* loss_history;
  int max_steps;
  smoe_adam_config adam;
};

inline StepScalarsArgs make_step_scalars_args(const smoe_fit_state& st, float* loss_out) {
  return StepScalarsArgs{st.step, st.scalars, loss_out, st.loss_history, st.max_steps, st.adam};
}

// The per-step Adam scalars of step t0 (Sec. VI-B): out[0] = the centre learning rate,
// decaying exponentially from lr_mu to lr_mu_final over total_steps; out[1], out[2] = the bias
// corrections 1 - beta1^(t0+1), 1 - beta2^(t0+1).  Computed once per step by one thread.
__device__ __forceinline__ void adam_step_scalars(const smoe_adam_config& ad, int t0,
                                                  float* __restrict__ out) {
  float lr_mu = ad.lr_mu;
  if (ad.total_steps > 0 && ad.lr_mu > 0.0f && ad.lr_mu_final > 0.0f)
    lr_mu = ad.lr_mu * powf(ad.lr_mu_final / ad.lr_mu, (float)t0 / (float)ad.total_steps);
  out[0] = lr_mu;
  out[1] = 1.0f - powf(ad.beta1, (float)(t0 + 1));
  out[2] = 1.0f - powf(ad.beta2, (float)(t0 + 1));
}

}  // namespace smoe
