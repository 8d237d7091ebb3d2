// Binning on gfx950: per-kernel box and render record, per-block counting, ordering of the
// (block, kernel) pairs and block ranges (Sec. IV-B "geometry shader", Sec. IV-C "subset
// kernel selection for each block").
//
// Ordering.  The pairs are ordered by block id and, within a block, by kernel id: the
// order a stable LSD radix sort by block id gives the kernel-major pair list.  It is
// computed as a radix sort whose single digit is the whole block id (2^14 buckets at
// 2048^2): an atomic histogram of the digit, one exclusive scan of the histogram (which
// is also the block ranges), a scatter into the buckets, and a per-bucket sort of the
// kernel ids in LDS that restores the stable order the atomic scatter does not keep.
// This is four launches, where a two-pass 7-bit LSD sort would need seven or more, and
// every pass is integer work over at most a few MB, so launch latency -- not HBM
// bandwidth -- is what the design minimises.
#include "smoe_internal.h"

namespace smoe {
namespace {

// Output-pixel index range whose centres lie in [lo, hi] (output units), clamped to
// [0, n-1]; false when empty.  NaN inputs give an empty range.
__device__ __forceinline__ bool axis_range(float lo, float hi, int n, int& i0, int& i1) {
  const float a = ceilf(lo - 0.5f);
  const float b = floorf(hi - 0.5f);
  const float last = (float)(n - 1);
  if (!(a <= last) || !(b >= 0.0f)) return false;
  i0 = (a < 0.0f) ? 0 : (int)a;
  i1 = (b > last) ? n - 1 : (int)b;
  return i0 <= i1;
}

// One thread per kernel: box (binary32, as specified in the ABI), block rectangle, count,
// render record, and one atomic increment per covered block.
__global__ __launch_bounds__(128) void k_preprocess(int K, int C, int order,
                                                    const float* __restrict__ params, GridArgs g,
                                                    int4* __restrict__ tile_rects,
                                                    int32_t* __restrict__ counts,
                                                    float* __restrict__ records, int rs,
                                                    int32_t* __restrict__ tile_counts) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  const int ne = expert_floats(C, order);
  const float* p = params + (size_t)j * (6 + ne);
  const float mux = p[0], muy = p[1], l11 = p[2], l21 = p[3], l22 = p[4], rho = p[5];

  // Square box, half-side R = r sqrt(lambda_max(L L^T)).
  const float sxx = l11 * l11;
  const float sxy = l11 * l21;
  const float syy = l21 * l21 + l22 * l22;
  const float h = 0.5f * (sxx + syy);
  const float d = 0.5f * (sxx - syy);
  const float lam = h + sqrtf(d * d + sxy * sxy);
  const float R = g.r * sqrtf(lam);
  const float fs = (float)g.scale;
  const float X0 = (mux - R) * fs - (float)g.ox;
  const float X1 = (mux + R) * fs - (float)g.ox;
  const float Y0 = (muy - R) * fs - (float)g.oy;
  const float Y1 = (muy + R) * fs - (float)g.oy;
  int u0, u1, v0, v1;
  const bool ok = axis_range(X0, X1, g.W, u0, u1) && axis_range(Y0, Y1, g.H, v0, v1);
  int4 rc = ok ? make_int4(u0 >> 4, v0 >> 4, u1 >> 4, v1 >> 4) : make_int4(0, 0, -1, -1);
  tile_rects[j] = rc;
  counts[j] = ok ? (rc.z - rc.x + 1) * (rc.w - rc.y + 1) : 0;

  float* rec = records + (size_t)j * rs;
  const float i11 = 1.0f / l11;
  const float i22 = 1.0f / l22;
  rec[0] = mux;
  rec[1] = muy;
  rec[2] = i11;
  rec[3] = l21;
  rec[4] = i22;
  rec[5] = rho * kLog2e;
  rec[6] = l21 * i22;
  for (int i = 0; i < ne; ++i) rec[kRecExpert + i] = p[6 + i];
  for (int i = kRecExpert + ne; i < rs; ++i) rec[i] = 0.0f;

  if (!ok) return;
  for (int ty = rc.y; ty <= rc.w; ++ty)
    for (int tx = rc.x; tx <= rc.z; ++tx) atomicAdd(&tile_counts[ty * g.ntx + tx], 1);
}

// One workgroup: exclusive scan of the per-block counts into [begin, end) ranges, the total
// P and the overflow flag; resets the counters to serve as scatter cursors.  Each pass
// covers 16384 blocks: every thread holds 16 consecutive counts in registers (4 x int4
// loads, contiguous across the wave), the thread totals are scanned with wave shuffles and
// one exchange of the 16 wave totals through LDS, and a running carry links the passes.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 16;
__device__ __forceinline__ long long wave_incl_scan(long long x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const long long o = __shfl_up(x, off);
    if (lane >= off) x += o;
  }
  return x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan(int T, int32_t* __restrict__ tile_counts,
                                                       int2* __restrict__ ranges, int capacity,
                                                       int32_t* __restrict__ status) {
  __shared__ long long s_wave[kScanThreads / 64];
  __shared__ int s_max[kScanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  long long carry = 0;
  int mx_all = 0;
  // First pass over all blocks computes P (needed before any range is written, so that an
  // overflow writes every range empty); the second writes the ranges.
  for (int write = 0; write < 2; ++write) {
    const bool over = write && carry > (long long)capacity;
    long long run = 0;
    for (int base = 0; base < T; base += kScanThreads * kScanItems) {
      const int b = base + tid * kScanItems;
      int c[kScanItems];
      if (b + kScanItems <= T) {
        const int4* p4 = reinterpret_cast<const int4*>(tile_counts + b);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
          const int4 v = p4[q];
          c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) c[q] = (b + q < T) ? tile_counts[b + q] : 0;
      }
      long long sum = 0;
      int mx = 0;
#pragma unroll
      for (int q = 0; q < kScanItems; ++q) {
        sum += c[q];
        mx = max(mx, c[q]);
      }
      const long long incl = wave_incl_scan(sum, lane);
      if (lane == 63) s_wave[wave] = incl;
      for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
      if (lane == 0) s_max[wave] = mx;
      __syncthreads();
      long long wbase = 0, total = 0;
      for (int w = 0; w < kScanThreads / 64; ++w) {
        const long long t = s_wave[w];
        if (w < wave) wbase += t;
        total += t;
      }
      if (!write)
        for (int w = 0; w < kScanThreads / 64; ++w) mx_all = max(mx_all, s_max[w]);
      __syncthreads();
      if (write) {
        long long off = run + wbase + incl - sum;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
          if (b + q < T) {
            ranges[b + q] = over ? make_int2(0, 0) : make_int2((int)off, (int)(off + c[q]));
            tile_counts[b + q] = 0;
          }
          off += c[q];
        }
      }
      run += total;
    }
    if (!write) carry = run;
  }
  if (tid == 0) {
    status[0] = (int)min(carry, (long long)INT32_MAX);
    status[1] = carry > (long long)capacity ? 1 : 0;
    status[2] = mx_all;
    status[3] = 0;
  }
}

// One thread per kernel: append the kernel id to each covered block's bucket.
__global__ __launch_bounds__(128) void k_scatter(int K, const int4* __restrict__ tile_rects,
                                                 int ntx, const int2* __restrict__ ranges,
                                                 int32_t* __restrict__ cursors,
                                                 uint32_t* __restrict__ vals,
                                                 const int32_t* __restrict__ status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K || status[1] != 0) return;
  const int4 rc = tile_rects[j];
  for (int ty = rc.y; ty <= rc.w; ++ty)
    for (int tx = rc.x; tx <= rc.z; ++tx) {
      const int t = ty * ntx + tx;
      const int pos = atomicAdd(&cursors[t], 1);
      const int2 rg = ranges[t];
      if (rg.x + pos < rg.y) vals[rg.x + pos] = (uint32_t)j;
    }
}

// One wave per block: sort the bucket's kernel ids ascending (bitonic sort in LDS for runs of
// up to kSortRun ids, then merges of sorted runs in global memory for longer buckets), and
// write the block id keys.  Kernel ids within a bucket are distinct.
constexpr int kSortThreads = 64;
constexpr int kSortRun = 2048;
__global__ __launch_bounds__(kSortThreads) void k_sort_buckets(const int2* __restrict__ ranges,
                                                               uint32_t* __restrict__ vals,
                                                               uint32_t* __restrict__ vals_alt,
                                                               uint32_t* __restrict__ keys) {
  __shared__ uint32_t s[kSortRun];
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const int2 rg = ranges[t];
  const int n = rg.y - rg.x;
  if (n <= 0) return;
  for (int i = tid; i < n; i += kSortThreads) keys[rg.x + i] = (uint32_t)t;
  if (n == 1) return;
  uint32_t* seg = vals + rg.x;
  for (int c0 = 0; c0 < n; c0 += kSortRun) {
    const int m = min(kSortRun, n - c0);
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    for (int i = tid; i < p2; i += kSortThreads) s[i] = (i < m) ? seg[c0 + i] : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int i = tid; i < p2; i += kSortThreads) {
          const int ixj = i ^ jj;
          if (ixj > i) {
            const uint32_t a = s[i], c = s[ixj];
            const bool up = (i & k) == 0;
            if ((a > c) == up) {
              s[i] = c;
              s[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = tid; i < m; i += kSortThreads) seg[c0 + i] = s[i];
    __threadfence_block();
    __syncthreads();
  }
  if (n <= kSortRun) return;
  // Pairwise merges of sorted runs: an element's output position is its index in its own
  // run plus the number of smaller elements in the partner run.
  uint32_t* src = seg;
  uint32_t* dst = vals_alt + rg.x;
  for (int width = kSortRun; width < n; width <<= 1) {
    for (int i = tid; i < n; i += kSortThreads) {
      const int run = i / width;
      const int pair_lo = (run & ~1) * width;
      const bool left = (run & 1) == 0;
      const int o_lo = left ? min(n, pair_lo + width) : pair_lo;
      const int o_hi = left ? min(n, pair_lo + 2 * width) : pair_lo + width;
      const uint32_t v = src[i];
      int lo = o_lo, hi = o_hi;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (src[mid] < v) lo = mid + 1;
        else hi = mid;
      }
      dst[pair_lo + (i - run * width) + (lo - o_lo)] = v;
    }
    __threadfence_block();
    __syncthreads();
    uint32_t* tmp = src;
    src = dst;
    dst = tmp;
  }
  if (src != seg) {
    for (int i = tid; i < n; i += kSortThreads) seg[i] = src[i];
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

hipError_t launch_bin(const smoe_model& m, const GridArgs& g, const smoe_bins& b, hipStream_t s) {
  // Counters start from zero every call (a fill kernel rather than a memset node, so that
  // the step can be captured into a graph).
  k_fill_i32<<<cdiv(g.T, 256), 256, 0, s>>>(b.tile_counts, g.T, 0);
  if (m.K > 0) {
    k_preprocess<<<cdiv(m.K, 128), 128, 0, s>>>(m.K, m.C, m.order, m.params, g,
                                                 reinterpret_cast<int4*>(b.tile_rects), b.counts,
                                                 b.records, b.record_stride, b.tile_counts);
  }
  k_scan<<<1, kScanThreads, 0, s>>>(g.T, b.tile_counts, reinterpret_cast<int2*>(b.ranges),
                                    b.capacity, b.status);
  if (m.K > 0) {
    k_scatter<<<cdiv(m.K, 128), 128, 0, s>>>(m.K, reinterpret_cast<const int4*>(b.tile_rects),
                                             g.ntx, reinterpret_cast<const int2*>(b.ranges),
                                             b.tile_counts, b.vals, b.status);
  }
  k_sort_buckets<<<g.T, kSortThreads, 0, s>>>(reinterpret_cast<const int2*>(b.ranges), b.vals,
                                              b.vals_alt, b.keys);
  return hipGetLastError();
}

}  // namespace smoe
