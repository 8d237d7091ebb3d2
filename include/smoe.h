/*
 * smoe.h -- C ABI of the MI355X (gfx950) rasterized Steered Mixture of Experts library.
 *
 * The library evaluates the SMoE image regression of Eq. (3)-(4) -- K anisotropic 2D
 * Gaussian gates (Eq. 2) with Cholesky-factored covariances (Sec. VI-B) and mixing
 * weights, normalised per pixel into soft gates over constant or linear experts --
 * restricted per 16x16 block to the kernels whose bounding box covers the block
 * (Eq. 5, Sec. IV-B/IV-C), together with the gradient of the reconstruction loss with
 * respect to every kernel parameter, which drives an Adam fitting loop (Sec. VI-B).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers marked "device" are HIP device pointers; all buffers are owned by the
 *    caller.  The library allocates no device memory and keeps no global state besides
 *    the static workspace of smoe_render_noalloc (one array per GPU).
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*; NULL = the
 *    null stream) and returns a status.  Arguments are validated on the host before
 *    anything is launched; on SMOE_ERR_INVALID nothing was enqueued.
 *  - Coordinates are pixels, x = column, y = row; native pixel (c, r) has its centre at
 *    (c + 0.5, r + 0.5).  An output raster (smoe_grid) samples output pixel (u, v) at
 *    the native point (((ox + u) + 0.5) * inv_s, ((oy + v) + 0.5) * inv_s), where
 *    inv_s = 1/scale rounded to binary32 once: scale > 1 is super-resolution by
 *    re-sampling the continuous regression (Sec. II-B, Sec. VII-C).
 *  - Images are float32 [height][width][C] (channel-interleaved); per-pixel scalars
 *    are float32 [height][width].  Blocks (tiles) are the 16x16 blocks of the output grid
 *    of the raster's scale, aligned to multiples of 16 in the output coordinate (ox + u,
 *    oy + v): the raster's blocks are those its pixels touch, numbered row-major from the
 *    one holding pixel (0, 0); T = ntx * nty with ntx = floor((ox + width - 1)/16) -
 *    floor(ox/16) + 1 (rows alike), i.e. ceil(width/16) for a block-aligned origin.  Blocks
 *    at the edges of a window may hang over it; their outside pixels are not written.
 *  - Kernel parameter rows are float32 [K][NP], NP = 6 + C * (1 + 2 * order):
 *      materialized row: mu_x, mu_y, l11, l21, l22, rho, a[C], wx[C], wy[C]
 *      raw row:          mu_x, mu_y, s1,  l21, s2,  rho, a[C], wx[C], wy[C]
 *    L = [[l11, 0], [l21, l22]] (l11, l22 > 0) is the Cholesky factor of Sigma,
 *    s1 = ln l11, s2 = ln l22, rho = ln pi (Eq. 4), and the expert is
 *    m(x) = a + wx (x - mu_x) + wy (y - mu_y) (order 1) or m = a (order 0).
 *    Gradients are reported in the raw order (d/ds1 = l11 d/dl11, d/ds2 = l22 d/dl22).
 *  - Truncation rule (Eq. 5 with the ellipse discard of Sec. IV-B).  The model is a function
 *    of native coordinates, and so is its truncation: blocks are the 16x16 blocks of the
 *    native pixel grid, and kernel j's blocks are those its box covers on the native raster
 *    (blocks holding a native pixel centre inside the box) -- the square box of half-side
 *    R = r * sqrt(lambda_max(Sigma_j)) (side = major axis of the ellipse, Fig. 3b), or the
 *    tight box (SMOE_BOX_TIGHT).  Kernel j is a member at a sample
 *    point x iff x's native block (floor(x/16), floor(y/16)) is one of j's blocks, whatever
 *    raster x was sampled on: a render at any scale and window re-samples the one regression
 *    (Sec. II-B, VII-C).  With the default reading (SMOE_TRUNC_GRADIENT, below) a member
 *    takes part in the render iff binary32 holds its term, i.e. its exponent
 *    a = fma(q, -log2(e)/2, rho*log2(e)) is >= -125, and in the gradient iff moreover
 *    q_j(x) = |L_j^-1 (x - mu_j)|^2 <= r^2 (with SMOE_TRUNC_RENDER, q <= r^2 for both).
 *    Every decision is an exactly specified binary32 computation:
 *      i11 = 1/l11, i22 = 1/l22; dx = x - mu_x, dy = y - mu_y; z1 = dx*i11;
 *      z2 = (dy - l21*z1)*i22; q = z1*z1 + z2*z2 (each op rounded, no fma); q <= r*r;
 *      log2(e) = 1.44269504f; rho*log2(e) rounded once; a by one fused multiply-add;
 *      sxx = l11*l11, sxy = l11*l21, syy = l21*l21 + l22*l22;
 *      lam = (sxx+syy)/2 + sqrt(((sxx-syy)/2)^2 + sxy^2); R = r*sqrt(lam);
 *      native pixel centres in the box: c from ceil((mu_x - R) - 0.5) to
 *      floor((mu_x + R) - 0.5); native blocks of j: floor(c/16) of those (x/16 computed as
 *      x * 0.0625), empty if no centre lies inside; rows alike;
 *      sample point of output pixel u: x(u) = ((ox + u) + 0.5) * inv_s.
 *    The block lists of an output raster hold, per output block, every kernel one of whose
 *    native blocks holds a sample point of the block; at scale 1 and origin 0 these are the
 *    native raster's lists.  A native block is 16*scale output pixels and begins on a
 *    multiple of 16 of the output coordinate -- the binary32 sample coordinates included,
 *    over the whole accepted range of origins, sizes and scales -- so every point of an
 *    output block lies in one native block and every kernel of its list is a member there.
 *    Within a block, kernels are visited in increasing kernel id, which is also the
 *    summation order of every per-pixel sum (renders are bitwise reproducible).  One
 *    exception: smoe_render and smoe_render_batched split a list longer than 128 entries
 *    into four contiguous quarters, sum each in kernel order and add the four partial sums
 *    in quarter order (still a fixed order), so on such blocks they are not bitwise equal to
 *    the fit step's render, which sums every list whole.
 *  - A pixel where no kernel takes part renders 0 and receives no gradient.
 *  - A kernel row with a NaN or infinite parameter (after sharpening) covers no block: it
 *    takes part nowhere, so the other kernels render and fit exactly as without it, and
 *    receives a zero gradient.  The binning (and, in a fit, each Adam step) raises the
 *    non-finite status word for it; smoe_read_status() reports SMOE_ERR_NONFINITE.
 *
 * Status codes are negative on error.  Asynchronous conditions detected on the device
 * (pair-capacity overflow, non-finite parameters) are reported through the workspace status
 * words and read back with smoe_read_status(), so that a whole fit step stays free of host
 * syncs.
 */
#ifndef SMOE_H_
#define SMOE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smoe_status;
#define SMOE_OK 0
#define SMOE_ERR_INVALID (-1)   /* bad argument: nothing was launched */
#define SMOE_ERR_CAPACITY (-2)  /* pair capacity too small (from smoe_read_status) */
#define SMOE_ERR_HIP (-3)       /* a HIP launch or copy failed */
#define SMOE_ERR_TOO_LARGE (-4) /* raster needs more blocks than the workspace holds */
#define SMOE_ERR_NONFINITE (-5) /* a kernel row holds NaN or infinity (from smoe_read_status) */

#define SMOE_TILE 16

/* Materialized model (device, read-only). */
typedef struct smoe_model {
  int32_t K;            /* number of kernels, >= 0 */
  int32_t C;            /* channels, 1 or 3 */
  int32_t order;        /* 0 = constant experts, 1 = linear (steered) experts */
  const float* params;  /* device [K][NP] materialized rows */
} smoe_model;

/* Output raster. */
typedef struct smoe_grid {
  int32_t width, height;       /* output pixels, 1 .. 65536 each */
  int32_t scale;               /* integer upscale factor, 1 .. 64 */
  int32_t origin_x, origin_y;  /* raster origin in output pixels, |.| <= 2^22 */
  float radius;                /* Mahalanobis truncation radius r in [2^-30, 2^30]
                                  (3 = 98.9 % mass) */
  float sharpen;               /* native sharpening (Sec. II-B, VII): every kernel is rendered
                                  with its bandwidth divided by this factor, L -> L / f (the
                                  box and the truncation test follow); f > 0, 0 or 1 = none.
                                  Render and binning only: the backward and the fit step
                                  reject f != 1 */
  int32_t box;                 /* SMOE_BOX_SQUARE or SMOE_BOX_TIGHT (below) */
  int32_t mode;                /* SMOE_MODE_SMOE or SMOE_MODE_RBF (below) */
  int32_t trunc;               /* SMOE_TRUNC_GRADIENT (0) or SMOE_TRUNC_RENDER (below) */
} smoe_grid;

/* Where the ellipse test of the truncation rule applies (Sec. IV-B).
 * SMOE_TRUNC_GRADIENT (the default): the render takes every member of the point's block
 * list whose term pi K binary32 can hold (exponent >= -125, so the term is a normal number;
 * below that the FP32 term would be lost to underflow, and the uncut FP64 sum of the lists
 * differs from this rule only by such terms); pixels outside a kernel's ellipse q <= r^2 are
 * dropped from the gradient only, which is then the sum of the in-ellipse (pixel, kernel)
 * pairs' terms of the rendered loss's gradient, with the render's y and D.
 * SMOE_TRUNC_RENDER: a kernel takes part at a point iff it is a member there and q <= r^2,
 * in the render and in the gradient (the gradient is that of the rendered loss).  Pixels
 * that every ellipse has left render 0 and get no gradient, so a long fit can strand them.
 * Any other value is rejected.  rho must stay below 88 (pi finite in binary32). */
#define SMOE_TRUNC_GRADIENT 0
#define SMOE_TRUNC_RENDER 1

/* Regression modes.  SMOE_MODE_SMOE: the gated regression of Eq. (2)-(4),
 * y_c = sum_j m_jc(x) pi_j K_j(x) / D with D = sum_i pi_i K_i(x) (y = 0 where D = 0).
 * SMOE_MODE_RBF: the weighted sum of kernels of Eq. (1) (RBF networks, Gaussian
 * splatting), y_c = sum_j pi_j m_jc(x) K_j(x): the kernel weight of Eq. (1) is pi_j m_jc(x)
 * (a constant for order 0), with no normalisation, so a pixel no kernel reaches renders 0.
 * Both modes share the boxes, block lists, truncation rule, parameter layout and records,
 * and write D; the render, the backward and the fit step follow the mode.  Any other value
 * is rejected. */
#define SMOE_MODE_SMOE 0
#define SMOE_MODE_RBF 1

/* Kernel boxes (Sec. IV-B).  SMOE_BOX_SQUARE: the paper's square box of half-side
 * R = r sqrt(lambda_max).  SMOE_BOX_TIGHT: the axis-aligned box of half-widths
 * Rx = min(R, r |l11| (1 + 2^-10) + m), Ry = min(R, r sqrt(syy) (1 + 2^-10) + m) with
 * syy = l21 l21 + l22 l22 and m = (|mu_x| + |mu_y| + R) 2^-18, in binary32 in that order:
 * the extents of the r-ellipse along x and y, widened by a margin that covers the rounding
 * of the binary32 ellipse test and of the pixel coordinates.  Every point the ellipse test
 * accepts lies in the tight box, so with SMOE_TRUNC_RENDER images and losses are those of
 * the square box, bit for bit; only blocks the ellipse cannot reach
 * leave the block lists, and gradients are the same sums of fewer (zero-free) per-block
 * partials, grouped differently, so they agree up to that rounding.  With
 * SMOE_TRUNC_GRADIENT the render of the dropped blocks loses the kernel's far tail, so the
 * tight box is then a different (cheaper) rule.  Any other value is rejected. */
#define SMOE_BOX_SQUARE 0
#define SMOE_BOX_TIGHT 1

/* One raster of a batched call: an image of a batched fit, or one render request (the
 * model rows params[param_offset, param_offset + num_kernels) rendered on this raster).
 * Rasters are numbered consecutively: kernel_offset, tile_offset and pixel_offset are the
 * raster's first row in the per-kernel workspace arrays, first block in the global block
 * numbering, and first pixel in the concatenated images; smoe_segments_layout() sets them. */
typedef struct smoe_segment {
  int32_t width, height;       /* output pixels, 1 .. 65536 each */
  int32_t scale;               /* integer upscale factor, 1 .. 64 */
  int32_t origin_x, origin_y;  /* raster origin in output pixels, |.| <= 2^22 */
  int32_t num_kernels;         /* rows of this raster's model */
  int32_t param_offset;        /* first row of the model in the params array */
  int32_t kernel_offset;       /* set by smoe_segments_layout */
  int32_t tile_offset;         /* set by smoe_segments_layout */
  float sharpen;               /* as smoe_grid.sharpen (0 or 1 = none) */
  int64_t pixel_offset;        /* set by smoe_segments_layout */
} smoe_segment;

/* Host only: sets kernel_offset, tile_offset and pixel_offset of segs[0, n) to the running
 * sums of num_kernels, blocks and pixels, and returns the totals (any output may be NULL).
 * Fails with SMOE_ERR_INVALID on an invalid raster or if a total exceeds int32 (blocks,
 * kernels). */
smoe_status smoe_segments_layout(smoe_segment* segs, int32_t n, int32_t* total_kernels,
                                 int32_t* total_tiles, int64_t* total_pixels);

/* A batch of rasters sharing one parameter array, expert shape and truncation radius. */
typedef struct smoe_batch {
  int32_t C, order;                   /* as in smoe_model */
  const float* params;                /* device, materialized rows addressed by param_offset */
  int32_t num_params_rows;            /* rows in params (for validation) */
  int32_t num_segments;               /* >= 1 */
  const smoe_segment* segments;       /* device copy of the laid-out table */
  const smoe_segment* segments_host;  /* host copy of the same table */
  float radius;                       /* truncation radius, as in smoe_grid */
  int32_t box;                        /* SMOE_BOX_SQUARE or SMOE_BOX_TIGHT */
  int32_t mode;                       /* SMOE_MODE_SMOE or SMOE_MODE_RBF */
  int32_t trunc;                      /* SMOE_TRUNC_GRADIENT or SMOE_TRUNC_RENDER */
} smoe_batch;

/* Binning workspace: the block lists of Sec. IV-C and the scratch of the backward.
 * Laid out by smoe_bins_layout() inside one caller-allocated device buffer. */
typedef struct smoe_bins {
  int32_t K, C, order;     /* model shape the workspace was laid out for */
  int32_t max_tiles;       /* largest block count T a raster may have */
  int32_t capacity;        /* largest number of (block, kernel) pairs P */
  int32_t* tile_rects;     /* [K][4] output blocks (tx0, ty0, tx1, ty1); empty = (0, 0, -1, -1) */
  int32_t* native_rects;   /* [K][4] native blocks (bx0, by0, bx1, by1) clamped to those the
                              raster's sample points reach; empty = (0, 0, -1, -1) */
  int32_t* counts;         /* [K] blocks covered by each kernel */
  float* records;          /* [K][record_stride] per-kernel render records */
  int32_t record_stride;   /* floats per record */
  int32_t* tile_counts;    /* [max_tiles] per-block counters (scratch) */
  int32_t* ranges;         /* [max_tiles][2] [begin, end) of each block's list */
  uint32_t* keys;          /* [capacity] block id of each pair, ascending */
  uint32_t* vals;          /* [capacity] kernel id of each pair, ascending within a block */
  uint32_t* vals_alt;      /* [capacity] scratch for very long block lists */
  float* pair_grads;       /* [16 K + capacity][NP rounded up to a multiple of 4] per-(block,
                              kernel) gradient partials (the centre's two without their
                              expert-slope terms, which the gradient gather adds once per
                              kernel): the standalone backward's at the pair's list position;
                              the fit step's at row 16 j + q for block q (row-major in kernel
                              j's rectangle) when q < 16, else at row 16 K + the pair's bucket
                              slot (NULL in a render-only workspace) */
  float* tile_loss;        /* [max_tiles] per-block squared error */
  int32_t* status;         /* [8]: pairs needed P, overflow flag, longest list, non-finite
                              flag of the last binning, then internal words (the fit step's
                              counter copy and overflow flags, the non-finite flag; a binning
                              clears the last one, a fit keeps it from its first step on) */
} smoe_bins;

/* Bytes of workspace needed for the given shape and limits (host only). */
size_t smoe_bins_workspace_bytes(int32_t K, int32_t C, int32_t order, int32_t max_tiles,
                                 int32_t capacity);

/* Carves `workspace` (device, >= smoe_bins_workspace_bytes(...) bytes, 256-byte aligned)
 * into `out`.  Host only; nothing is launched and the memory is not touched. */
smoe_status smoe_bins_layout(smoe_bins* out, void* workspace, size_t bytes, int32_t K, int32_t C,
                             int32_t order, int32_t max_tiles, int32_t capacity);

/* A render-only workspace: the same layout without the per-pair gradient partials
 * (pair_grads = NULL), for callers that bin and render but never run the backward -- a
 * serving loop.  smoe_render_backward and smoe_fit_step reject such bins with
 * SMOE_ERR_INVALID.  Host only, as smoe_bins_workspace_bytes / smoe_bins_layout. */
size_t smoe_render_workspace_bytes(int32_t K, int32_t C, int32_t order, int32_t max_tiles,
                                   int32_t capacity);
smoe_status smoe_render_workspace_layout(smoe_bins* out, void* workspace, size_t bytes, int32_t K,
                                         int32_t C, int32_t order, int32_t max_tiles,
                                         int32_t capacity);

/* Binning (Sec. IV-B, IV-C): per-kernel box (smoe_grid.box) -> block rectangle and count, the
 * per-kernel render record, then the (block, kernel) pairs ordered by block and, within a
 * block, by kernel id, and each block's [begin, end) range.  The order is the one a
 * stable radix sort by block id of the kernel-major pair list gives.  If P exceeds
 * bins->capacity the status words record the needed P and the overflow flag, every
 * range is written empty, and later calls on these bins render zeros and skip updates. */
smoe_status smoe_bin(const smoe_model* model, const smoe_grid* grid, smoe_bins* bins,
                     void* stream);

/* Forward render (Eq. 3-5): image (device [H][W][C]) and, if denom != NULL, the
 * per-pixel gate denominator D = sum_j pi_j K_j (device [H][W]) that the backward reuses.
 * If target (device [H][W][C]) and loss_out (device float[1]) are both non-NULL, also
 * writes loss_out[0] = mean over H*W*C of (image - target)^2.  `bins` must come from
 * smoe_bin() with the same model and grid. */
smoe_status smoe_render(const smoe_model* model, const smoe_grid* grid, const smoe_bins* bins,
                        float* image, float* denom, const float* target, float* loss_out,
                        void* stream);

/* Backward (adjoint of smoe_render; the parameters are fitted by descending the
 * reconstruction error's gradient, Sec. II-A and VI-B, with the out-of-ellipse pixels of a
 * kernel's blocks discarded from its gradient, Sec. IV-B): writes grads (device [K][NP], raw
 * order) = dL/dparams, recomputing every gate from the saved image and denom.  Exactly one of
 * grad_image (device [H][W][C], upstream dL/dimage) and target (device [H][W][C]: L = the
 * mean squared error of image against target) must be non-NULL.  Gradients are
 * written, not accumulated.  Uses bins->pair_grads as scratch. */
smoe_status smoe_render_backward(const smoe_model* model, const smoe_grid* grid,
                                 const smoe_bins* bins, const float* image, const float* denom,
                                 const float* grad_image, const float* target, float* grads,
                                 void* stream);

/* Batched binning and render: every segment of `batch` is binned into one workspace (laid
 * out for K = total kernels, max_tiles >= total blocks) and rendered into the concatenated
 * images (device [total pixels][C]) and denominators ([total pixels], may be NULL), exactly
 * as smoe_bin + smoe_render of each raster alone would.  One launch per stage serves all
 * segments (render requests of a serving loop, images of a batched fit). */
smoe_status smoe_bin_batched(const smoe_batch* batch, smoe_bins* bins, void* stream);
smoe_status smoe_render_batched(const smoe_batch* batch, const smoe_bins* bins, float* images,
                                float* denoms, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): smoe_bin + smoe_render of one raster with
 * no caller workspace.  The binning workspace lives in a static device array of the library
 * (64 MiB per GPU, held until the process ends), laid out as a render-only workspace with
 * max_tiles = the raster's blocks and the largest pair capacity that fits.  The caller
 * passes the model, the raster and the outputs only: image (device [H][W][C]), denom
 * (device [H][W], may be NULL) and status_out (device int32[4], may be NULL: receives the
 * status words P needed, overflow flag, longest list, non-finite flag).  Images are bitwise those of
 * smoe_bin + smoe_render with the same model and grid.  Returns SMOE_ERR_TOO_LARGE when the
 * per-kernel and per-block arrays alone exceed the static array; a pair overflow is
 * reported through status_out[1] (the image is then zeros), never by a host sync.  Nothing
 * is allocated, and no hipMemset is issued.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams or threads) race and must be
 * serialised by the caller.  The library sets up a device's array on its first call there. */
smoe_status smoe_render_noalloc(const smoe_model* model, const smoe_grid* grid, float* image,
                                float* denom, int32_t* status_out, void* stream);

/* raw -> materialized rows (l11 = exp(s1), l22 = exp(s2), the rest copied), device. */
smoe_status smoe_materialize(int32_t K, int32_t C, int32_t order, const float* raw,
                             float* model, void* stream);

/* Adam settings of a fit (Sec. VI-B).  The centre learning rate decays exponentially
 * from lr_mu to lr_mu_final over total_steps: lr_mu(t) = lr_mu*(lr_mu_final/lr_mu)^(t/total);
 * the Cholesky parameters (s1, l21, s2), rho and the experts use fixed rates. */
typedef struct smoe_adam_config {
  float lr_mu, lr_mu_final, lr_chol, lr_rho, lr_expert;
  float beta1, beta2, eps;
  int32_t total_steps;
} smoe_adam_config;

/* State of one fit.  Every pointer is device memory owned by the caller; `raw`, `adam_m`,
 * `adam_v` must be initialised (m = v = 0 for a fresh fit) and `model` must hold
 * smoe_materialize(raw) before the first step; `step` holds the number of completed
 * steps (0 for a fresh fit). */
typedef struct smoe_fit_state {
  int32_t K, C, order;
  smoe_grid grid;            /* the target raster: scale 1, origin 0 */
  smoe_adam_config adam;
  float* raw;                /* [K][NP] raw parameters, updated in place */
  float* adam_m;             /* [K][NP] */
  float* adam_v;             /* [K][NP] */
  float* model;              /* [K][NP] materialized rows of `raw` */
  float* grads;              /* [K][NP] gradient of the last step (raw order), or NULL */
  float* image;              /* [H][W][C] render of the last step that wrote it */
  float* denom;              /* [H][W] */
  float* loss_history;       /* [max_steps] loss before each update, or NULL */
  int32_t max_steps;
  int32_t prepared;          /* host flag: 1 when the workspace already holds the block
                                counts and ranges of `model` (each step leaves them for the
                                next); set 0 for a fresh fit, a new workspace, or after
                                changing raw/model outside smoe_fit_step */
  int32_t write_render;      /* 1: the step writes its render to image and denom; 0: it
                                leaves them as they are (the loss, the gradient and the
                                update need neither, so a fit loop skips 16 B per pixel of
                                stores on all but the steps whose render it wants) */
  int32_t* step;             /* [1] completed steps */
  float* scalars;            /* [4] per-step scratch (the step's Adam learning rate and bias
                                corrections) */
  /* Batched fit (num_segments > 0): num_segments images fitted together, each with its own
   * kernels, as independent fits stepped in lock-step (the loss is the sum of the images'
   * MSEs, so every image's gradient is its own).  Segments laid out by
   * smoe_segments_layout with scale 1, origin 0 and param_offset == kernel_offset; target,
   * image and denom are the concatenated images; K = total kernels; of `grid` only the radius,
   * the box, the mode and the truncation are used. */
  int32_t num_segments;
  const smoe_segment* segments;       /* device copy, or NULL for one image */
  const smoe_segment* segments_host;  /* host copy, or NULL */
  smoe_bins bins;            /* laid out for (K, C, order) and all blocks */
} smoe_fit_state;

/* One fit iteration (Sec. VI-B: Adam on every kernel parameter, the centre rate decaying
 * exponentially; the rasterized forward and backward of Sec. IV) on `stream` with no host
 * synchronisation: binning, forward render
 * with the fused squared-error loss, backward, then per kernel the deterministic
 * reduction of its block partials, the Adam update of the raw row and its
 * re-materialization.  The step runs as three kernels: the scatter, which computes each
 * kernel's box from its model row and puts the (block, kernel) pairs into block buckets; one
 * kernel that per 16x16 block orders its bucket, renders the block and runs its backward;
 * and Adam, which also records the loss and writes the next step's render records (so the
 * first step, state->prepared == 0, computes those first and then sets
 * state->prepared = 1).  The workspace's pair storage is used as fixed-width
 * buckets: each of the T blocks gets floor(bins.capacity / T) entries, so the capacity must
 * cover T times the longest block list; with W = floor(capacity / T) and 16 + W rounded up
 * to a power of two 2^b, the total kernel count must stay below 2^(32 - b) (each bucket entry
 * holds the kernel id and the row of its gradient partial in 32 bits), else the call returns
 * SMOE_ERR_TOO_LARGE.  A fuller
 * bucket is a capacity overflow: the step
 * changes nothing (the step counter included) and smoe_read_status() reports it, with
 * status[0] = T x the longest list and status[2] = the longest list.  loss_out (device
 * float[1], may be NULL) and loss_history[step] receive the loss before the update.  grads
 * holds the last step's gradient; image and denom its render and denominator when
 * write_render is set. */
smoe_status smoe_fit_step(smoe_fit_state* state, const float* target, float* loss_out,
                          void* stream);

/* smoe_fit_step with HIP events recorded on `stream` at the stage boundaries, for timing:
 * stage_events[0] before binning, [1] after binning (scan and scatter), [2] after the fused
 * per-block render + backward kernel, [3] after Adam (with the next step's binning front).
 * stage_events is a host array of 4 hipEvent_t; NULL entries are not recorded. */
smoe_status smoe_fit_step_timed(smoe_fit_state* state, const float* target, float* loss_out,
                                void* const* stage_events, void* stream);

/* Diagnostic (not part of a fit step): counts, over the raster's in-image pixels, the
 * (pixel, kernel) pairs a render tests -- every kernel of the pixel's block list -- and the
 * pairs that take part (q <= r^2).  out2 is device uint64[2] = (tested, active) and is
 * overwritten.  Uses atomics; the counts are exact integers. */
smoe_status smoe_pair_stats(const smoe_model* model, const smoe_grid* grid,
                            const smoe_bins* bins, uint64_t* out2, void* stream);

/* Diagnostic (not part of the method): the issue-rate probe behind the compute roofline's
 * peak.  Launches `workgroups` workgroups of 256 threads; each thread runs 8 independent
 * chains of `iters` iterations of one binary32 instruction -- kind 0: fma with all operands in
 * vector registers, 1: fma reading a scalar register, 2: v_exp_f32 -- and writes
 * their sum to out (device float[workgroups * 256]).  The caller times the launch on
 * `stream`; the kernel issues workgroups * 4 * iters * 8 wave64 instructions of that kind.
 * 1 <= iters, 1 <= workgroups <= 2^20, kind in 0..2, else SMOE_ERR_INVALID. */
smoe_status smoe_issue_probe(int32_t kind, int32_t iters, int32_t workgroups, float* out,
                             void* stream);

/* Reporting: out (device float[max(1, num_segments)]) = each image's MSE at the state's last
 * fit step. */
smoe_status smoe_fit_segment_losses(const smoe_fit_state* state, float* out, void* stream);

/* Multi-model fusion (Sec. V-C, Eq. (10)-(11)): the estimate at each pixel is the mean of the
 * predictions of every window model that covers it.  Windows of window x window pixels are
 * shifted by the displacement d (window % d == 0) along both axes; along an axis of n pixels
 * window k covers [max(0, (k+1)d - window), min(n, (k+1)d)), so the first window starts
 * window - d pixels before the image, windows are clipped to it, and every pixel lies in
 * exactly m = window/d windows per axis (H = m^2 hypotheses; window 16 and d = 16, 8, 4, 2
 * give H = 1, 4, 16, 64).
 * window_images (device float) holds every window's render, concatenated in window order --
 * rows of windows top to bottom, each row left to right -- each window's clipped pixels
 * row-major with C channels interleaved: m^2 * width * height * C floats in all (the layout
 * of smoe_render_batched over the windows' rasters in that order).  image (device float
 * [height][width][C]) receives, per pixel and channel, the binary32 sum of the m^2 covering
 * windows in (window row, window column) order divided by m^2: one fixed order, no atomics,
 * bitwise reproducible.  C is 1 or 3; 1 <= width, height <= 65536; 1 <= window <= 1024.
 * SMOE_ERR_INVALID on a bad argument (nothing launched). */
smoe_status smoe_fuse_windows(const float* window_images, int32_t C, int32_t width,
                              int32_t height, int32_t window, int32_t displacement,
                              float* image, void* stream);

/* Synchronises `stream`, copies the status words (P needed, overflow flag, longest list,
 * non-finite flag) into host out4 (may be NULL) and returns SMOE_ERR_CAPACITY after an
 * overflow, else SMOE_ERR_NONFINITE when the last binning -- or, in a fit workspace, any step
 * of the fit so far -- met a kernel row with a NaN or infinite parameter. */
smoe_status smoe_read_status(const smoe_bins* bins, int32_t* out4, void* stream);

/* Name and description of the HIP error behind this thread's last SMOE_ERR_HIP ("no
 * error" if none).  The string is owned by the library and valid until the next failing
 * call on the thread. */
const char* smoe_last_error(void);

/* Library version, e.g. 100 for 0.1.0. */
int32_t smoe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMOE_H_ */
