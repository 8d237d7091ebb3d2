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
// Every pass is integer work over a few MB, so the design minimises launches, not bytes.
// The fit step uses fixed-width buckets instead (k_scatter_fixed): no histogram and no scan,
// the bucket of block t is entries [t W, t W + W) of the pair storage.
#include "device_common.h"

namespace smoe {
namespace {

// The kernel that group g of a binning kernel's lanes (kPreLanes, kScatterLanes) takes: every
// 8th of 128 consecutive kernel ids (a bijection on each complete run of 128; the ids past
// the last one keep their order).  Neighbouring ids are neighbours in the image (the grid
// initialisation's order, which the kernels keep as they move), so a wave's counter and
// cursor atomics stay within a few blocks; spreading them over eight times as many ids keeps
// that locality while fewer atomics of one instruction meet on the same counter, where they
// serialise.  Any order gives the same counts and, up to the order inside a bucket, which
// the sorts that follow remove, the same buckets.
__device__ __forceinline__ int binning_kernel(int g, int K) {
  return (g | 127) < K ? (g & ~127) + ((g & 15) << 3) + ((g >> 4) & 7) : g;
}

// Four lanes per kernel row (so that a wave covers 16 kernels and a launch has four times the
// waves to hide its loads): every lane of the quad reads the row and computes the
// output-block and native-block rectangles; lane 0 writes them and the count, lane q the
// q-th float4 of the render record, and (tile_counts not null) lane q adds one to the counts
// of the kernel's covered blocks q, q + 4, ... (row-major).  A row with a NaN or infinite
// parameter covers no block (it takes part nowhere) and sets the non-finite status word.
constexpr int kPreLanes = 4;
__global__ __launch_bounds__(256) void k_preprocess(int C, int order,
                                                    const float* __restrict__ params, Segs S,
                                                    int4* __restrict__ tile_rects,
                                                    int4* __restrict__ native_rects,
                                                    int32_t* __restrict__ counts,
                                                    float* __restrict__ records, int rs,
                                                    int32_t* __restrict__ tile_counts,
                                                    int32_t* __restrict__ status) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = gid / kPreLanes, lq = gid % kPreLanes;
  if (g >= S.K) return;
  const int j = binning_kernel(g, S.K);
  const SegGrid sg = seg_of_kernel(S, j);
  const int ne = expert_floats(C, order);
  const float* p = params + (size_t)(sg.param_offset + (j - sg.kernel_offset)) * (6 + ne);
  // native sharpening: the raster sees L / f (a correctly rounded binary32 division)
  float l11 = p[2], l21 = p[3], l22 = p[4];
  if (sg.sharpen != 1.0f) {
    l11 = l11 / sg.sharpen;
    l21 = l21 / sg.sharpen;
    l22 = l22 / sg.sharpen;
  }
  bool finite = __builtin_isfinite(l11) && __builtin_isfinite(l21) && __builtin_isfinite(l22);
  for (int k = 0; k < 6 + ne; ++k) finite = finite && __builtin_isfinite(p[k]);
  KernelRects kr;
  if (finite) {
    kr = kernel_rects(p[0], p[1], l11, l21, l22, sg, S.r, S.box, S.trunc);
  } else {
    kr.tile = kr.native = make_int4(0, 0, -1, -1);
  }
  const int4 rc = kr.tile;
  if (lq == 0) {
    tile_rects[j] = rc;
    native_rects[j] = kr.native;
    counts[j] = rect_count(rc);
    if (!finite) status[kNonfinite] = 1;
  }
  if (lq < rs / 4) write_record_quad(records + (size_t)j * rs, p, ne, lq, l11, l21, l22);
  if (tile_counts) count_blocks(rc, sg, tile_counts, lq, kPreLanes);
}

constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_scan(int T, int32_t* __restrict__ tile_counts,
                                                       int2* __restrict__ ranges, int capacity,
                                                       int32_t* __restrict__ status) {
  __shared__ int s_begin[16 * kScanThreads];
  __shared__ long long s_tot[kScanThreads / 64];
  block_scan_ranges<kScanThreads>(T, tile_counts, ranges, capacity, status, s_begin, s_tot);
}

// Four lanes per kernel: lane q appends the kernel id to the buckets of the kernel's
// covered blocks q, q + 4, ... (row-major inside its block rectangle), so the cursor
// atomics of one kernel run in parallel rather than one after another.
constexpr int kScatterLanes = 4;
__global__ __launch_bounds__(256) void k_scatter(Segs S, const int4* __restrict__ tile_rects,
                                                 const int2* __restrict__ ranges,
                                                 int32_t* __restrict__ cursors,
                                                 uint32_t* __restrict__ vals,
                                                 const int32_t* __restrict__ status) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = gid / kScatterLanes, q0 = gid % kScatterLanes;
  if (g >= S.K || status[1] != 0) return;
  const int j = binning_kernel(g, S.K);
  const int4 rc = tile_rects[j];
  const int n = rect_count(rc);
  if (n == 0) return;
  const SegGrid sg = seg_of_kernel(S, j);
  const int w = rc.z - rc.x + 1;
  for (int q = q0; q < n; q += kScatterLanes) {
    const int t = sg.tile_offset + (rc.y + q / w) * sg.ntx + rc.x + q % w;
    const int pos = atomicAdd(&cursors[t], 1);
    const int2 rg = ranges[t];
    if (rg.x + pos < rg.y) vals[rg.x + pos] = (uint32_t)j;
  }
}

// The fit step's scatter into fixed-width buckets: entry t W + c of the pair storage, c the
// block's cursor, receives (kernel id << shift) | low, where low names the row the block's
// partial row of the kernel will be written to and read back from, so that no later pass has
// to search the sorted lists: low = q, the block's row-major index in the kernel's rectangle,
// for q < kSlots (row kSlots j + q), else kSlots + c (row kSlots K + t W + c).  A bucket that
// fills up sets the step's overflow flag (status word kStepFlags + parity of the step
// counter) and drops the entry -- the step then changes nothing.  The cursors start at zero
// (the fused render resets them).  The kernel's block rectangle comes from its model row
// (kernel_rects, the binning's own rule; a row with a NaN or infinite parameter covers no
// block) and is stored with its count for the step's Adam kernel, which gathers the
// kernel's partial rows over it.  Thread 0 copies the step counter into the status words
// and writes the step's Adam scalars, for the step's later kernels.
__global__ __launch_bounds__(256) void k_scatter_fixed(Segs S, const float* __restrict__ model,
                                                       int np, int4* __restrict__ tile_rects,
                                                       int32_t* __restrict__ counts,
                                                       int32_t* __restrict__ cursors,
                                                       uint32_t* __restrict__ vals, int width,
                                                       int shift, int32_t* __restrict__ status,
                                                       const int32_t* __restrict__ step,
                                                       smoe_adam_config adam,
                                                       float* __restrict__ scalars) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int t0 = step[0];
  if (gid == 0) {
    status[kStepShadow] = t0;
    adam_step_scalars(adam, t0, scalars);
  }
  const int g = gid / kScatterLanes, q0 = gid % kScatterLanes;
  if (g >= S.K) return;  // (whole groups of kScatterLanes lanes: the shuffles stay inside one)
  const int j = binning_kernel(g, S.K);
  const SegGrid sg = seg_of_kernel(S, j);
  // every lane of the kernel's group reads the geometry; lane q0 also checks parameters
  // 5 + q0, 5 + q0 + kScatterLanes, ... for finiteness
  const float* p = model + (size_t)j * np;
  const float mux = p[0], muy = p[1], l11 = p[2], l21 = p[3], l22 = p[4];
  bool finite = __builtin_isfinite(mux) && __builtin_isfinite(muy) && __builtin_isfinite(l11) &&
                __builtin_isfinite(l21) && __builtin_isfinite(l22);
  for (int k = 5 + q0; k < np; k += kScatterLanes) finite = finite && __builtin_isfinite(p[k]);
  int bad = finite ? 0 : 1;
  static_assert(kScatterLanes == 4, "the finiteness vote spans a quad");
  bad |= __shfl_xor(bad, 1);
  bad |= __shfl_xor(bad, 2);
  int4 rc = make_int4(0, 0, -1, -1);
  if (!bad) rc = kernel_rects(mux, muy, l11, l21, l22, sg, S.r, S.box, S.trunc).tile;
  const int n = rect_count(rc);
  if (q0 == 0) {
    tile_rects[j] = rc;
    counts[j] = n;
  }
  if (n == 0) return;
  const int w = rc.z - rc.x + 1;
  for (int q = q0; q < n; q += kScatterLanes) {
    const int t = sg.tile_offset + (rc.y + q / w) * sg.ntx + rc.x + q % w;
    const int pos = atomicAdd(&cursors[t], 1);
    if (pos < width) {
      const uint32_t low = q < kSlots ? (uint32_t)q : (uint32_t)(kSlots + pos);
      vals[(size_t)t * width + pos] = ((uint32_t)j << shift) | low;
    } else {
      status[kStepFlags + (t0 & 1)] = 1;
    }
  }
}

// One wave per block: sort the bucket ascending, write the block-id keys, reset the
// block's cursor.
constexpr int kSortRun = 2048;
__global__ __launch_bounds__(64) void k_sort_buckets(const int2* __restrict__ ranges,
                                                     uint32_t* __restrict__ vals,
                                                     uint32_t* __restrict__ vals_alt,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ cursors) {
  __shared__ uint32_t s[kSortRun];
  const int t = blockIdx.x;
  const int2 rg = ranges[t];
  const int n = rg.y - rg.x;
  if (threadIdx.x == 0) cursors[t] = 0;
  if (n <= 0) return;
  for (int i = threadIdx.x; i < n; i += 64) keys[rg.x + i] = (uint32_t)t;
  if (n <= 64) rank_sort64(vals + rg.x, n, s, nullptr);
  else sort_bucket(vals + rg.x, vals_alt + rg.x, n, s, kSortRun);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The binning's first kernel: zero the per-block counters and the non-finite flag.
__global__ void k_fill_counts(int32_t* __restrict__ counts, int n, int32_t* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counts[i] = 0;
  if (i == 0) status[kNonfinite] = 0;
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

hipError_t launch_count(int C, int order, const float* params, const Segs& S,
                        const smoe_bins& b, hipStream_t s) {
  // Counters and the non-finite flag start from zero (a fill kernel rather than a memset
  // node, so that the step can be captured into a graph).
  k_fill_counts<<<cdiv(S.T, 256), 256, 0, s>>>(b.tile_counts, S.T, b.status);
  if (S.K > 0) {
    k_preprocess<<<cdiv((long long)S.K * kPreLanes, 256), 256, 0, s>>>(C, order, params, S,
                                                 reinterpret_cast<int4*>(b.tile_rects),
                                                 reinterpret_cast<int4*>(b.native_rects), b.counts,
                                                 b.records, b.record_stride, b.tile_counts,
                                                 b.status);
  }
  return hipGetLastError();
}

hipError_t launch_scan(const Segs& S, const smoe_bins& b, hipStream_t s) {
  k_scan<<<1, kScanThreads, 0, s>>>(S.T, b.tile_counts, reinterpret_cast<int2*>(b.ranges),
                                    b.capacity, b.status);
  return hipGetLastError();
}

hipError_t launch_prepare_fit(int C, int order, const float* params, const Segs& S,
                              const smoe_bins& b, hipStream_t s) {
  k_fill_i32<<<cdiv(S.T, 256), 256, 0, s>>>(b.tile_counts, S.T, 0);
  // A fresh fit starts from clear status words (P, overflow, longest list, step shadow, the
  // overflow flags and the non-finite flag), whatever the workspace held before.
  k_fill_i32<<<1, 64, 0, s>>>(b.status, 8, 0);
  if (S.K > 0) {
    k_preprocess<<<cdiv((long long)S.K * kPreLanes, 256), 256, 0, s>>>(C, order, params, S,
                                                 reinterpret_cast<int4*>(b.tile_rects),
                                                 reinterpret_cast<int4*>(b.native_rects), b.counts,
                                                 b.records, b.record_stride, nullptr, b.status);
  }
  return hipGetLastError();
}

hipError_t launch_scatter_fixed(const Segs& S, const smoe_bins& b, const float* model, int np,
                                int width, int shift, const int32_t* step,
                                const smoe_adam_config& adam, float* scalars, hipStream_t s) {
  k_scatter_fixed<<<max(1, cdiv((long long)S.K * kScatterLanes, 256)), 256, 0, s>>>(
      S, model, np, reinterpret_cast<int4*>(b.tile_rects), b.counts, b.tile_counts, b.vals,
      width, shift, b.status, step, adam, scalars);
  return hipGetLastError();
}

hipError_t launch_scatter(const Segs& S, const smoe_bins& b, hipStream_t s) {
  if (S.K > 0) {
    k_scatter<<<cdiv((long long)S.K * kScatterLanes, 256), 256, 0, s>>>(
        S, reinterpret_cast<const int4*>(b.tile_rects), reinterpret_cast<const int2*>(b.ranges),
        b.tile_counts, b.vals, b.status);
  }
  return hipGetLastError();
}

hipError_t launch_copy_status(const smoe_bins& b, int32_t* out4, hipStream_t s) {
  k_copy_i32<<<1, 64, 0, s>>>(b.status, out4, 4);
  return hipGetLastError();
}

hipError_t launch_bin(int C, int order, const float* params, const Segs& S, const smoe_bins& b,
                      hipStream_t s) {
  hipError_t e = launch_count(C, order, params, S, b, s);
  if (e == hipSuccess) e = launch_scan(S, b, s);
  if (e == hipSuccess) e = launch_scatter(S, b, s);
  if (e != hipSuccess) return e;
  k_sort_buckets<<<S.T, 64, 0, s>>>(reinterpret_cast<const int2*>(b.ranges), b.vals, b.vals_alt,
                                    b.keys, b.tile_counts);
  return hipGetLastError();
}

}  // namespace smoe
