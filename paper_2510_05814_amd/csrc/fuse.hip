// Multi-model fusion of block-overlapping window models (Sec. V-C, Eq. (10)-(11)) on gfx950.
//
// Along an axis of n pixels, window k of size w shifted by the displacement d covers
// [max(0, (k+1)d - w), min(n, (k+1)d)): the first window starts w - d pixels before the
// image, and every pixel x lies in exactly m = w/d windows per axis, k = floor(x/d) ...
// floor(x/d) + m - 1.  The window renders arrive concatenated in window order (rows of
// windows top to bottom, each row left to right), each window's clipped pixels row-major with
// C channels interleaved.  Since every row of windows holds m n_x pixels per image row, the
// start of window (ky, kx) is prefix_y(ky) m n_x + len_y(ky) prefix_x(kx), with prefix(k) the
// pixels of windows 0 .. k-1 of an axis, in closed form.
//
// One thread per output pixel sums the m^2 windows that cover it in (ky, kx) order, in
// binary32, and divides by m^2 (correctly rounded): a gather with one fixed order and no
// atomics, so the fused image is bitwise reproducible.  The kernel is HBM bound: every window
// pixel is read once (m^2 W H C floats), W H C floats are written.
#include "smoe_internal.h"

namespace smoe {
namespace {

struct FuseAxis {
  int n, d, w, m;

  __device__ int start(int k) const {
    const int e = (k + 1) * d - w;
    return e > 0 ? e : 0;
  }
  __device__ int len(int k) const { return min(n, (k + 1) * d) - start(k); }
  // sum over i = 1 .. k of min(n, i d) - max(0, i d - w)
  __device__ long long prefix(int k) const {
    const long long q = n / d, kk = k;
    long long s = kk <= q ? d * (kk * (kk + 1) / 2) : d * (q * (q + 1) / 2) + (kk - q) * n;
    if (kk > m) s -= d * (kk * (kk + 1) / 2 - (long long)m * (m + 1) / 2) - (long long)w * (kk - m);
    return s;
  }
};

template <int C>
__global__ __launch_bounds__(256) void k_fuse_windows(const float* __restrict__ win, FuseAxis ax,
                                                      FuseAxis ay, float hyp,
                                                      float* __restrict__ out) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= ax.n || y >= ay.n) return;
  const long long row_pixels = (long long)ax.m * ax.n;
  const int kx0 = x / ax.d, ky0 = y / ay.d;
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0f;
  for (int ky = ky0; ky < ky0 + ay.m; ++ky) {
    const long long hy = ay.len(ky);
    const long long base = ay.prefix(ky) * row_pixels;
    const long long dy = y - ay.start(ky);
    for (int kx = kx0; kx < kx0 + ax.m; ++kx) {
      const long long wx = ax.len(kx);
      const long long p = base + hy * ax.prefix(kx) + dy * wx + (x - ax.start(kx));
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] += win[p * C + c];
    }
  }
  const long long o = ((long long)y * ax.n + x) * C;
#pragma unroll
  for (int c = 0; c < C; ++c) out[o + c] = acc[c] / hyp;
}

}  // namespace

hipError_t launch_fuse_windows(const float* windows, int C, int width, int height, int window,
                               int d, float* image, hipStream_t s) {
  const int m = window / d;
  const FuseAxis ax{width, d, window, m}, ay{height, d, window, m};
  const dim3 grid((width + 63) / 64, (height + 3) / 4);
  const float hyp = (float)((long long)m * m);
  if (C == 1) k_fuse_windows<1><<<grid, 256, 0, s>>>(windows, ax, ay, hyp, image);
  else k_fuse_windows<3><<<grid, 256, 0, s>>>(windows, ax, ay, hyp, image);
  return hipGetLastError();
}

}  // namespace smoe
