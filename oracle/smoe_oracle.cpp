// Plain CPU oracle for the rasterized Steered Mixture of Experts (R-SMoE) image model.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or load this
// file's library; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do.  It shares no source with the HIP implementation.
//
// What it computes, straight from the definitions (every loop visits ALL K kernels at
// every pixel it evaluates; no binning, tiling or reordering is used to get a value):
//
//   * Steered Gaussian kernel, Eq. (2):  K_j(x) = exp(-1/2 (x-mu_j)^T Sigma_j^-1 (x-mu_j)),
//     with Sigma_j = L_j L_j^T and L_j = [[l11, 0], [l21, l22]] its Cholesky factor
//     (Sec. VI-B).  q_j(x) = |L_j^-1 (x - mu_j)|^2 by forward substitution.
//   * Soft gates, Eq. (4): w_j = pi_j K_j / sum_i pi_i K_i, with pi_j = exp(rho_j).
//   * SMoE regression, Eq. (3): y(x) = sum_j m_j(x) w_j(x); experts are constant
//     m_j = a_j (Sec. II-A) or linear ("steered") m_j(x) = a_j + W_j (x - mu_j).
//   * Rasterized truncation, Eq. (5) with the discard rule of Sec. IV-B.  The model is a
//     function of native image coordinates, so the blocks are the 16x16 blocks of the
//     native pixel grid: a kernel's blocks are the native blocks its square bounding box
//     (side = major axis of its confidence ellipse, Fig. 3b) covers -- with the block lists
//     deciding the render, those holding a native pixel centre inside the box (the lists of
//     the native raster); with the ellipse test deciding, those the box overlaps, so that
//     every point inside the ellipse is a member at any scale -- and the kernel belongs to the
//     list of a sample point x iff x's native block
//     (floor(x / 16), per axis) is one of them -- whatever raster (scale, window) x is
//     sampled on, so super-resolution and windows re-sample one regression (Sec. II-B,
//     VII-C).  Pixels of a kernel's blocks outside its ellipse q_j(x) <= r^2 are discarded
//     in the gradient.  Two readings (trunc): 1 = as the section states, the render takes
//     every kernel of the block's list and the ellipse test only removes (point, kernel)
//     pairs from the gradient, which is then the sum of the in-ellipse pairs' terms of the
//     rendered loss's gradient (with the render's D and y) -- a listed term is rendered
//     whenever binary32 can hold it: its exponent rho log2(e) - q log2(e) / 2, rounded as
//     the GPU forms it, is >= -125 (so pi K >= 2^-125 is a normal binary32 number); 0 = the
//     ellipse test applies to the render too (kernel j takes part at x iff x's block is one
//     of its blocks AND q_j(x) <= r^2), so the gradient is exactly the rendered loss's.
//     Every conjunct is a discrete decision evaluated in exactly specified IEEE binary32
//     arithmetic (this file is built with -ffp-contract=off; the exponent's one fused
//     multiply-add is written as std::fmaf), the same precision as the GPU kernels, so that
//     both take the same decisions.  Every continuous quantity (exp, sums, y, gradients) is
//     FP64.
//   * Optionally (box = 1) a tight axis-aligned box instead of the square one: half-widths
//     r sqrt(Sigma_xx) and r sqrt(Sigma_yy), the extents of the r-ellipse along x and y,
//     each widened by a small margin that covers the rounding of the binary32 ellipse test
//     and capped at the square box.  Every pixel the ellipse test accepts inside the square
//     box lies inside the widened tight box, so with the ellipse test in the render the
//     model's values are unchanged; only blocks that the ellipse cannot reach leave the
//     lists.  (When the block lists alone decide the render, the tight box drops far tails
//     from it.)
//   * Optionally (rbf = 1) the weighted sum of kernels of Eq. (1) (RBF networks, Gaussian
//     splatting) instead of the gates: y(x) = sum_j pi_j m_j(x) K_j(x), the kernel weight of
//     Eq. (1) being pi_j m_j(x); no normalisation.  Same kernels, truncation and parameters.
//   * The untruncated ("global") model of Sec. III-B: every kernel at every pixel.
//   * Block lists of Sec. IV-C: per 16x16 block of an output raster, the kernels one of
//     whose native blocks holds a sample point of the block, in increasing kernel id.  At
//     native resolution (scale 1, origin 0) these are the kernels whose box covers the block.
//   * For the truncation report: the block-list sum without any cut (every listed kernel at
//     every point of its blocks).
//   * The analytic gradient of the mean-squared reconstruction error (Sec. II-A: the
//     parameters are adjusted to minimise the error between reconstruction and image)
//     with respect to every raw kernel parameter, and Adam (Sec. VI-B).
//
// Readings of points the paper leaves open (the design notes list them all):
//   r is a parameter (3 in the workloads; the 99 % ellipse of Sec. IV-B would be 3.035);
//   q == r^2 is inside; a pixel with no participating kernel renders 0 and has no
//   gradient; the loss is the mean over H*W*C; pixel (u, v) is sampled at native
//   coordinate ((o + u) + 0.5) / s with 1/s rounded to binary32 once.
//
// Parameter rows (double, NP = 6 + C*(1 + 2*order) per kernel):
//   materialized: mu_x, mu_y, l11, l21, l22, rho, a[C], wx[C], wy[C]
//   raw:          mu_x, mu_y, s1,  l21, s2,  rho, a[C], wx[C], wy[C]   (l11 = e^s1, l22 = e^s2)
// Gradients are always reported in the raw order (d/ds1 = l11 d/dl11, d/ds2 = l22 d/dl22).
//
// Parity status: every function here is pinned by CPU tests (closed forms, library
// routines, brute force, invariants, finite differences) except oracle_fit beyond one
// step, whose trajectory is "parity unpinned" (FP32 and FP64 Adam trajectories
// legitimately diverge).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct Grid {
  int W, H;     // output raster size in pixels
  int s;        // integer upscale factor (1 = native resolution)
  int ox, oy;   // raster origin in output pixels
  float r;      // Mahalanobis truncation radius
  int box;      // 0: square box of Sec. IV-B; 1: tight axis-aligned box
  int rbf;      // 0: gated SMoE regression, Eq. (2)-(4); 1: weighted sum of kernels, Eq. (1)
  int trunc;    // 1: the ellipse test applies to the gradient only; 0: render and gradient
  // Blocks: the 16x16 blocks of the output grid of this scale, aligned to multiples of 16 in
  // the output coordinate o + u; the raster's blocks are those its pixels touch, numbered
  // from the one holding its first pixel.
  int ntx() const { return first_block(ox + W - 1) - first_block(ox) + 1; }
  int nty() const { return first_block(oy + H - 1) - first_block(oy) + 1; }
  static int first_block(int g) { return (int)std::floor(g / 16.0); }
  // The first output pixel (window coordinate, may be negative) of block t along an axis.
  static int block_start(int t, int o) { return 16 * (first_block(o) + t) - o; }
};

int num_params(int C, int order) { return 6 + C * (1 + 2 * order); }

// ------------------------------------------------------------------------------------
// The binary32 part of the rule.
// ------------------------------------------------------------------------------------

// Native sampling coordinate of output pixel index u along one axis.
float coord32(int u, int o, int s) {
  const float inv_s = 1.0f / (float)s;
  return ((float)(o + u) + 0.5f) * inv_s;
}

// Native 16x16 block index of a native coordinate, floor(x / 16) (x * 2^-4 is exact).
float native_block(float x) { return std::floor(x * 0.0625f); }

constexpr float kLog2eF = 1.44269504088896340736f;

struct Rect32 {
  bool empty;
  float bx0, bx1, by0, by1;  // native block rect (integer-valued), clamped to the raster's
  int tx0, tx1, ty0, ty1;    // output block rect of the raster (inclusive)
};

// The native blocks [b0, b1] of a box's extent [lo, hi] along one axis.  centres: the blocks
// holding a native pixel centre c + 0.5 inside it, c from ceil(lo - 0.5) to floor(hi - 0.5) --
// the blocks the box covers on the native raster (scale 1, origin 0), the block lists that
// decide the render.  Otherwise: the blocks the box overlaps, floor(lo / 16) to
// ceil(hi / 16) - 1 -- every block holding a point of the box (no sample point lies on a
// block boundary), so that with the ellipse test deciding the render every point inside the
// ellipse is a member at any scale.  False when empty (or NaN).
bool native_axis(float lo, float hi, bool centres, float* b0, float* b1) {
  if (centres) {
    const float a = std::ceil(lo - 0.5f);
    const float b = std::floor(hi - 0.5f);
    if (!(a <= b)) return false;
    *b0 = native_block(a);
    *b1 = native_block(b);
    return true;
  }
  *b0 = native_block(lo);
  *b1 = std::ceil(hi * 0.0625f) - 1.0f;
  return *b0 <= *b1;
}

// The output blocks [t0, t1] of an axis of n sample points (origin o, scale s; blocks of 16
// aligned to multiples of 16 in o + u, Grid) holding a point whose native block lies in
// [b0, b1]: every block is scanned, each by its first and last point inside the raster (the
// native block index does not decrease along the axis).  The native rect is clamped to the
// blocks the raster's points reach.  False when none does.
bool output_axis(float* b0, float* b1, int n, int o, int s, int* t0, int* t1) {
  const float first = native_block(coord32(0, o, s));
  const float last = native_block(coord32(n - 1, o, s));
  if (*b1 < first || *b0 > last) return false;
  *b0 = std::max(*b0, first);
  *b1 = std::min(*b1, last);
  *t0 = -1;
  *t1 = -2;
  const int nt = Grid::first_block(o + n - 1) - Grid::first_block(o) + 1;
  for (int t = 0; t < nt; ++t) {
    const int u0 = std::max(0, Grid::block_start(t, o));
    const int u1 = std::min(n - 1, Grid::block_start(t, o) + 15);
    const float a = native_block(coord32(u0, o, s));
    const float b = native_block(coord32(u1, o, s));
    if (a <= *b1 && b >= *b0) {
      if (*t0 < 0) *t0 = t;
      *t1 = t;
    }
  }
  return *t0 >= 0;
}

// Square box centred on mu with half-side R = r * sqrt(lambda_max(Sigma)): its side is
// the major axis of the r-ellipse (Fig. 3b).  lambda_max of the symmetric 2x2 matrix
// by the closed form  (sxx+syy)/2 + sqrt(((sxx-syy)/2)^2 + sxy^2).  The box selects native
// blocks; the raster's output blocks follow from them.
// native_only: the native blocks alone, unclamped (no raster; output rect left empty).
Rect32 kernel_rect32(float mux, float muy, float l11, float l21, float l22, const Grid& g,
                     bool native_only = false) {
  const float sxx = l11 * l11;
  const float sxy = l11 * l21;
  const float syy = l21 * l21 + l22 * l22;
  const float h = 0.5f * (sxx + syy);
  const float d = 0.5f * (sxx - syy);
  const float lam = h + std::sqrt(d * d + sxy * sxy);
  const float R = g.r * std::sqrt(lam);
  float Rx = R, Ry = R;
  if (g.box == 1) {
    // The ellipse's x extent is r |l11| (z1 = dx / l11 and q >= z1^2); its y extent is
    // r sqrt(syy) (dy = l21 z1 + l22 z2, Cauchy-Schwarz).  The margin: 2^-10 relative,
    // plus 2^-18 of the coordinates' magnitude for the roundings of the pixel centre and
    // of the box edges.
    const float m = (std::fabs(mux) + std::fabs(muy) + R) * 0x1p-18f;
    Rx = std::fmin(R, g.r * std::fabs(l11) * 1.0009765625f + m);
    Ry = std::fmin(R, g.r * std::sqrt(syy) * 1.0009765625f + m);
  }
  Rect32 rc{};
  const bool centres = g.trunc == 1;
  rc.empty = !(native_axis(mux - Rx, mux + Rx, centres, &rc.bx0, &rc.bx1) &&
               native_axis(muy - Ry, muy + Ry, centres, &rc.by0, &rc.by1));
  if (native_only) {
    rc.tx0 = rc.ty0 = 0;
    rc.tx1 = rc.ty1 = -1;
    return rc;
  }
  rc.empty = rc.empty || !(output_axis(&rc.bx0, &rc.bx1, g.W, g.ox, g.s, &rc.tx0, &rc.tx1) &&
                           output_axis(&rc.by0, &rc.by1, g.H, g.oy, g.s, &rc.ty0, &rc.ty1));
  if (rc.empty) {
    rc.tx0 = rc.ty0 = 0;
    rc.tx1 = rc.ty1 = -1;
    rc.bx0 = rc.by0 = 0.0f;
    rc.bx1 = rc.by1 = -1.0f;
  }
  return rc;
}

// q = |L^-1 (x - mu)|^2 as the exact binary32 sequence: reciprocals of the diagonal, then
// z1 = dx/l11, z2 = (dy - l21 z1)/l22.
float q32(float x, float y, float mux, float muy, float l11, float l21, float l22) {
  const float i11 = 1.0f / l11;
  const float i22 = 1.0f / l22;
  const float dx = x - mux;
  const float dy = y - muy;
  const float z1 = dx * i11;
  const float t = l21 * z1;
  const float w = dy - t;
  const float z2 = w * i22;
  return z1 * z1 + z2 * z2;
}

// Whether binary32 holds the term pi K = 2^arg with arg = rho log2(e) - q log2(e) / 2
// formed as the GPU forms it (one rounded product, one fused multiply-add): arg >= -125.
bool representable32(float q, float rho) {
  const float rl = rho * kLog2eF;
  const float arg = std::fmaf(q, -0.5f * kLog2eF, rl);
  return arg >= -125.0f;
}

// ------------------------------------------------------------------------------------
// FP64 model.
// ------------------------------------------------------------------------------------

// Which terms a point takes: RULE_ELLIPSE (block member and q <= r^2: the gradient, and the
// render with the ellipse test in it), RULE_LISTS (block member and a representable term:
// the render when the block lists decide it), RULE_UNCUT (block member: the report).
enum Rule { RULE_ELLIPSE, RULE_LISTS, RULE_UNCUT };

struct Model {
  int K, C, order, NP;
  const double* p;  // [K][NP] materialized
  std::vector<Rect32> rect;
  std::vector<float> f32;  // [K][6] binary32 view: mux, muy, l11, l21, l22, rho

  // native_only: boxes on the native grid alone (evaluation at arbitrary points).
  Model(int K_, int C_, int order_, const double* p_, const Grid& g, bool native_only = false)
      : K(K_), C(C_), order(order_), NP(num_params(C_, order_)), p(p_), rect(K_), f32(6 * (size_t)K_) {
    for (int j = 0; j < K; ++j) {
      const double* r = p + (size_t)j * NP;
      float* f = &f32[6 * (size_t)j];
      for (int k = 0; k < 6; ++k) f[k] = (float)r[k];
      rect[j] = kernel_rect32(f[0], f[1], f[2], f[3], f[4], g, native_only);
    }
  }

  // Whether kernel j takes part at the sample point (x32, y32) under `rule`.  Only native
  // quantities enter: the point's native block and the kernel's native blocks.
  bool participates(int j, float x32, float y32, Rule rule, float r2) const {
    const Rect32& rc = rect[j];
    if (rc.empty) return false;
    const float bx = native_block(x32), by = native_block(y32);
    if (bx < rc.bx0 || bx > rc.bx1 || by < rc.by0 || by > rc.by1) return false;
    if (rule == RULE_UNCUT) return true;
    const float* f = &f32[6 * (size_t)j];
    const float q = q32(x32, y32, f[0], f[1], f[2], f[3], f[4]);
    return rule == RULE_ELLIPSE ? q <= r2 : representable32(q, f[5]);
  }
};

// Per-(pixel, kernel) quantities of the FP64 model.
struct Term {
  double dx, dy, z1, z2, e;
};

inline Term term(const double* r, double x, double y) {
  Term t;
  t.dx = x - r[0];
  t.dy = y - r[1];
  t.z1 = t.dx / r[2];
  t.z2 = (t.dy - r[3] * t.z1) / r[4];
  const double q = t.z1 * t.z1 + t.z2 * t.z2;
  t.e = std::exp(r[5] - 0.5 * q);  // pi_j K_j(x)
  return t;
}

// Expert value m_jc at offset (dx, dy) from the kernel centre.
inline double expert(const double* r, int C, int order, int c, double dx, double dy) {
  double m = r[6 + c];
  if (order == 1) m += r[6 + C + c] * dx + r[6 + 2 * C + c] * dy;
  return m;
}

// y(x) and D(x) = sum_j pi_j K_j(x) at the native point (x32, y32) over the participating
// kernels (truncated: 0 = all K, the global model of Sec. III-B; 1 = the truncation rule of
// the reading; 2 = every kernel of the point's block list, uncut); y = N / D (Eq. 2-4) or,
// in the RBF mode, y = N (Eq. 1), with N_c = sum_j pi_j K_j m_jc.  Nothing here depends on
// the raster the point was sampled on.
void eval_point(const Model& M, const Grid& g, int truncated, float x32, float y32, double* y,
                double* D) {
  const float r2 = g.r * g.r;
  const Rule rule = truncated == 2 ? RULE_UNCUT : (g.trunc == 1 ? RULE_LISTS : RULE_ELLIPSE);
  const double x = (double)x32, yy = (double)y32;
  double Dsum = 0.0;
  std::vector<double> N(M.C, 0.0);
  for (int j = 0; j < M.K; ++j) {
    if (truncated && !M.participates(j, x32, y32, rule, r2)) continue;
    const double* r = M.p + (size_t)j * M.NP;
    const Term t = term(r, x, yy);
    Dsum += t.e;
    for (int c = 0; c < M.C; ++c) N[c] += t.e * expert(r, M.C, M.order, c, t.dx, t.dy);
  }
  *D = Dsum;
  for (int c = 0; c < M.C; ++c) y[c] = g.rbf ? N[c] : ((Dsum > 0.0) ? N[c] / Dsum : 0.0);
}

// The value at output pixel (u, v): the model at the pixel's native sample point.
void eval_pixel(const Model& M, const Grid& g, int truncated, int u, int v, double* y, double* D) {
  eval_point(M, g, truncated, coord32(u, g.ox, g.s), coord32(v, g.oy, g.s), y, D);
}

template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  if (threads <= 1 || n <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i, 0);
    return;
  }
  threads = (int)std::min<int64_t>(threads, n);
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&, t] {
      for (;;) {
        const int64_t i = next.fetch_add(1);
        if (i >= n) break;
        f(i, t);
      }
    });
  }
  for (auto& th : pool) th.join();
}

// Accumulates the gradient contribution of pixel (u, v) into G (raw-parameter order,
// rows indexed through `slot`, -1 = not requested).  g[c] = dL/dy_c at this pixel.
void grad_pixel(const Model& M, const Grid& g, int u, int v, const double* gy_in,
                const double* y, double D, const int32_t* slot, double* G) {
  if (!(D > 0.0)) return;  // no participating kernel: y is the constant 0
  const float x32 = coord32(u, g.ox, g.s);
  const float y32 = coord32(v, g.oy, g.s);
  const float r2 = g.r * g.r;
  const double x = (double)x32, yy = (double)y32;
  const int C = M.C, NP = M.NP;
  for (int j = 0; j < M.K; ++j) {
    const int32_t sj = slot ? slot[j] : j;
    if (sj < 0) continue;
    if (!M.participates(j, x32, y32, RULE_ELLIPSE, r2)) continue;
    const double* r = M.p + (size_t)j * NP;
    const Term t = term(r, x, yy);
    // w = dy_c/dm_jc: the gate w_j(x) of Eq. (4), or pi_j K_j(x) in the RBF sum of Eq. (1).
    const double w = g.rbf ? t.e : t.e / D;
    // Gs = dL/de_j / (w / e_j), with e_j = pi_j K_j: gated, dL/de_j = sum_c g_c (m_jc - y_c)/D;
    // RBF, dL/de_j = sum_c g_c m_jc.  Either way dL/drho_j = e_j dL/de_j = w Gs.
    double Gs = 0.0;
    for (int c = 0; c < C; ++c)
      Gs += gy_in[c] * (expert(r, C, M.order, c, t.dx, t.dy) - (g.rbf ? 0.0 : y[c]));
    const double Hh = w * Gs;
    double* out = G + (size_t)sj * NP;
    out[5] += Hh;
    // Expert parameters: dy_c/dm_jc = w_j.
    double ex = 0.0, ey = 0.0;  // sum_c g_c w dm_jc/d(dx), d(dy)
    for (int c = 0; c < C; ++c) {
      const double gw = gy_in[c] * w;
      out[6 + c] += gw;
      if (M.order == 1) {
        out[6 + C + c] += gw * t.dx;
        out[6 + 2 * C + c] += gw * t.dy;
        ex += gw * r[6 + C + c];
        ey += gw * r[6 + 2 * C + c];
      }
    }
    // Gate geometry: dL/dq = -Hh/2; dq/dz = 2 z; z2 depends on z1 through -l21/l22.
    const double bz2 = -Hh * t.z2;
    const double bz1 = -Hh * t.z1 - bz2 * r[3] / r[4];
    const double bdx = bz1 / r[2] + ex;
    const double bdy = bz2 / r[4] + ey;
    out[0] -= bdx;                       // dx = x - mu_x
    out[1] -= bdy;
    out[2] += -bz1 * t.z1;               // l11 dL/dl11, since dz1/dl11 = -z1/l11
    out[3] += -bz2 * t.z1 / r[4];        // dz2/dl21 = -z1/l22
    out[4] += -bz2 * t.z2;               // l22 dL/dl22, since dz2/dl22 = -z2/l22
  }
}

}  // namespace

extern "C" {

int oracle_num_params(int C, int order) { return num_params(C, order); }

// Per-kernel boxes and the per-block kernel lists of Sec. IV-C (trunc: the reading, which
// decides how a box selects native blocks).
//   tile_rects   [K][4] = output blocks (tx0, ty0, tx1, ty1), empty = (0, 0, -1, -1)
//   native_rects [K][4] = native blocks (bx0, by0, bx1, by1) clamped to the blocks the
//                         raster's sample points reach, empty = (0, 0, -1, -1) (may be NULL)
//   counts       [K]    = number of output blocks in the kernel's rect
//   keys/vals  [capacity] = (block id, kernel id) pairs ordered by block, then kernel id
//   ranges     [T][2] = [begin, end) of each block's list in keys/vals
// Returns the total number of pairs P (written only up to capacity).
int64_t oracle_bin(int K, int C, int order, const double* model, int W, int H, int s, int ox,
                   int oy, float r, int box, int trunc, int32_t* tile_rects, int32_t* native_rects,
                   int32_t* counts,
                   int64_t capacity, uint32_t* keys, uint32_t* vals, int32_t* ranges) {
  const Grid g{W, H, s, ox, oy, r, box, 0, trunc};
  const Model M(K, C, order, model, g);
  const int ntx = g.ntx(), T = g.ntx() * g.nty();
  std::vector<std::vector<uint32_t>> lists(T);
  for (int j = 0; j < K; ++j) {
    const Rect32& rc = M.rect[j];
    int32_t* tr = tile_rects + 4 * (size_t)j;
    tr[0] = rc.tx0; tr[1] = rc.ty0; tr[2] = rc.tx1; tr[3] = rc.ty1;
    if (native_rects) {
      int32_t* nr = native_rects + 4 * (size_t)j;
      nr[0] = (int32_t)rc.bx0; nr[1] = (int32_t)rc.by0;
      nr[2] = (int32_t)rc.bx1; nr[3] = (int32_t)rc.by1;
    }
    counts[j] = rc.empty ? 0 : (rc.tx1 - rc.tx0 + 1) * (rc.ty1 - rc.ty0 + 1);
    if (rc.empty) continue;
    for (int ty = rc.ty0; ty <= rc.ty1; ++ty)
      for (int tx = rc.tx0; tx <= rc.tx1; ++tx) lists[ty * ntx + tx].push_back((uint32_t)j);
  }
  int64_t P = 0;
  for (int t = 0; t < T; ++t) {
    if (ranges) { ranges[2 * t] = (int32_t)std::min<int64_t>(P, INT32_MAX); }
    for (uint32_t j : lists[t]) {
      if (P < capacity) { keys[P] = (uint32_t)t; vals[P] = j; }
      ++P;
    }
    if (ranges) { ranges[2 * t + 1] = (int32_t)std::min<int64_t>(P, INT32_MAX); }
  }
  return P;
}

// Renders y [npix][C] and D [npix] at the listed output pixels (pix [npix][2] = (u, v));
// pix == NULL renders the whole raster in row-major order (npix ignored).  truncated: 0 =
// every kernel (Sec. III-B), 1 = the truncation rule, 2 = the uncut block lists.
void oracle_render(int K, int C, int order, const double* model, int W, int H, int s, int ox,
                   int oy, float r, int box, int rbf, int trunc, int truncated, int64_t npix,
                   const int32_t* pix,
                   double* y,
                   double* D, int threads) {
  const Grid g{W, H, s, ox, oy, r, box, rbf, trunc};
  const Model M(K, C, order, model, g);
  const int64_t n = pix ? npix : (int64_t)W * H;
  parallel_for(n, threads, [&](int64_t i, int) {
    const int u = pix ? pix[2 * i] : (int)(i % W);
    const int v = pix ? pix[2 * i + 1] : (int)(i / W);
    eval_pixel(M, g, truncated, u, v, y + (size_t)i * C, D + i);
  });
}

// The model at arbitrary binary32 native points pts [npts][2] = (x, y), independent of any
// raster: the kernel boxes are taken on the native grid (a raster of scale 1 and origin 0
// spanning every native block), so the rule sees only the points and the model.
void oracle_render_points(int K, int C, int order, const double* model, float r, int box,
                          int rbf, int trunc, int truncated, int64_t npts, const float* pts,
                          double* y, double* D, int threads) {
  const Grid g{1, 1, 1, 0, 0, r, box, rbf, trunc};
  const Model M(K, C, order, model, g, true);
  parallel_for(npts, threads, [&](int64_t i, int) {
    eval_point(M, g, truncated, pts[2 * i], pts[2 * i + 1], y + (size_t)i * C, D + i);
  });
}

// Loss and gradient of the truncated model on the full output raster (W, H, s, ox, oy).
//   target [H][W][C]: loss = mean((y - t)^2), dL/dy = 2 (y - t) / (H W C)
//   or grad_y [H][W][C]: upstream dL/dy (target ignored, loss reported as 0)
//   sel [nsel]: kernel ids whose gradients are wanted (NULL = all K, nsel ignored);
//     only pixels in the requested kernels' blocks are visited, which is exact because
//     a kernel contributes nothing outside its blocks; the loss is then not available.
//   grads [nsel or K][NP] raw-parameter order, overwritten.
// Returns the loss (NaN in grad_y mode or with a kernel subset).
double oracle_loss_grad(int K, int C, int order, const double* model, int W, int H, int s, int ox,
                        int oy, float r, int box, int rbf, int trunc, const double* target,
                        const double* grad_y,
                        int nsel,
                        const int32_t* sel, double* grads, int threads) {
  const Grid g{W, H, s, ox, oy, r, box, rbf, trunc};
  const Model M(K, C, order, model, g);
  const int NP = M.NP;
  const int nout = sel ? nsel : K;
  std::vector<int32_t> slot;
  std::vector<uint8_t> need;  // pixel mask
  if (sel) {
    slot.assign(K, -1);
    need.assign((size_t)W * H, 0);
    for (int i = 0; i < nsel; ++i) {
      const int j = sel[i];
      slot[j] = i;
      const Rect32& rc = M.rect[j];
      if (rc.empty) continue;
      const int v0 = std::max(0, Grid::block_start(rc.ty0, oy));
      const int v1 = std::min(H, Grid::block_start(rc.ty1, oy) + 16);
      const int u0 = std::max(0, Grid::block_start(rc.tx0, ox));
      const int u1 = std::min(W, Grid::block_start(rc.tx1, ox) + 16);
      for (int v = v0; v < v1; ++v)
        for (int u = u0; u < u1; ++u) need[(size_t)v * W + u] = 1;
    }
  }
  threads = std::max(1, threads);
  std::vector<std::vector<double>> Gt(threads, std::vector<double>((size_t)nout * NP, 0.0));
  std::vector<double> loss_row(H, 0.0);
  const double inv_n = 1.0 / ((double)W * H * C);
  parallel_for(H, threads, [&](int64_t v, int tid) {
    std::vector<double> y(C), gy(C);
    double lr = 0.0;
    for (int u = 0; u < W; ++u) {
      const size_t p = (size_t)v * W + u;
      const bool want = !sel || need[p];
      if (!want) continue;
      double D;
      eval_pixel(M, g, 1, u, (int)v, y.data(), &D);
      for (int c = 0; c < C; ++c) {
        if (grad_y) {
          gy[c] = grad_y[p * C + c];
        } else {
          const double d = y[c] - target[p * C + c];
          lr += d * d;
          gy[c] = 2.0 * d * inv_n;
        }
      }
      if (want) grad_pixel(M, g, u, (int)v, gy.data(), y.data(), D, sel ? slot.data() : nullptr,
                           Gt[tid].data());
    }
    loss_row[v] = lr;
  });
  std::fill(grads, grads + (size_t)nout * NP, 0.0);
  for (int t = 0; t < threads; ++t)
    for (size_t i = 0; i < (size_t)nout * NP; ++i) grads[i] += Gt[t][i];
  double loss = 0.0;
  for (int v = 0; v < H; ++v) loss += loss_row[v];
  // The loss needs every pixel; with a kernel subset only some were evaluated.
  if (grad_y || sel) return std::nan("");
  return loss * inv_n;
}

// Raw parameters -> materialized model (l11 = e^s1, l22 = e^s2, the rest copied).
void oracle_materialize(int K, int C, int order, const double* raw, double* model) {
  const int NP = num_params(C, order);
  for (int j = 0; j < K; ++j) {
    const double* a = raw + (size_t)j * NP;
    double* m = model + (size_t)j * NP;
    for (int k = 0; k < NP; ++k) m[k] = a[k];
    m[2] = std::exp(a[2]);
    m[4] = std::exp(a[4]);
  }
}

// Learning rates of one step.  Groups: centres (columns 0-1), Cholesky (2-4), mixing
// weight rho (5), experts (6..).  The centre rate decays exponentially from lr_mu to
// lr_mu_final over total_steps (Sec. VI-B): lr_mu(t) = lr_mu * (lr_mu_final/lr_mu)^(t/total).
void oracle_step_lrs(int step_index, int total_steps, double lr_mu, double lr_mu_final,
                     double lr_chol, double lr_rho, double lr_expert, double* out4) {
  double f = 1.0;
  if (total_steps > 0 && lr_mu > 0.0 && lr_mu_final > 0.0)
    f = std::pow(lr_mu_final / lr_mu, (double)step_index / (double)total_steps);
  out4[0] = lr_mu * f;
  out4[1] = lr_chol;
  out4[2] = lr_rho;
  out4[3] = lr_expert;
}

// One Adam update (Kingma & Ba, with bias correction) of K rows of NP parameters.
// t is the 1-based step number; lrs4 = per-group rates as from oracle_step_lrs.
void oracle_adam(int K, int C, int order, double* p, const double* g, double* m, double* v, int t,
                 const double* lrs4, double beta1, double beta2, double eps) {
  const int NP = num_params(C, order);
  const double bc1 = 1.0 - std::pow(beta1, t);
  const double bc2 = 1.0 - std::pow(beta2, t);
  for (int j = 0; j < K; ++j) {
    for (int k = 0; k < NP; ++k) {
      const size_t i = (size_t)j * NP + k;
      const double lr = k < 2 ? lrs4[0] : (k < 5 ? lrs4[1] : (k == 5 ? lrs4[2] : lrs4[3]));
      m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
      v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
      const double mhat = m[i] / bc1;
      const double vhat = v[i] / bc2;
      p[i] -= lr * mhat / (std::sqrt(vhat) + eps);
    }
  }
}

// Full fit: `steps` iterations of materialize -> loss/gradient -> Adam, from raw0.
// Writes the loss before each update into loss_hist [steps] and the final raw params.
void oracle_fit(int K, int C, int order, const double* raw0, int W, int H, float r, int box,
                int rbf, int trunc,
                const double* target, int steps, int total_steps, double lr_mu,
                double lr_mu_final, double lr_chol, double lr_rho, double lr_expert,
                double beta1, double beta2, double eps, double* loss_hist, double* raw_out,
                int threads) {
  const int NP = num_params(C, order);
  const size_t n = (size_t)K * NP;
  std::vector<double> raw(raw0, raw0 + n), model(n), g(n), m(n, 0.0), v(n, 0.0);
  double lrs[4];
  for (int it = 0; it < steps; ++it) {
    oracle_materialize(K, C, order, raw.data(), model.data());
    loss_hist[it] = oracle_loss_grad(K, C, order, model.data(), W, H, 1, 0, 0, r, box, rbf, trunc, target,
                                     nullptr,
                                     0, nullptr, g.data(), threads);
    oracle_step_lrs(it, total_steps, lr_mu, lr_mu_final, lr_chol, lr_rho, lr_expert, lrs);
    oracle_adam(K, C, order, raw.data(), g.data(), m.data(), v.data(), it + 1, lrs, beta1, beta2,
                eps);
  }
  std::memcpy(raw_out, raw.data(), n * sizeof(double));
}

}  // extern "C"
