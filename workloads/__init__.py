"""Seeded synthetic inputs for the rasterized SMoE hot path.

This module produces *inputs only*: target images and the initial kernel
parameters that a fit starts from.  It contains none of the model's
arithmetic (no gates, no truncation rule, no gradients), so both the GPU
path and the CPU oracle may use it without sharing any of the method.

The paper's own workloads are natural photographs (Kodak 768x512 and DIV2K
around 1060x768, Sec. VI-A); those datasets are not used here.  The images
below are synthetic stand-ins with the piecewise-smooth structure the model
is built for (flat regions, ramps and sharp edges, Sec. II), at the sizes of
the workloads this project measures.

Parameter layouts (float32, one row per kernel, NP = 6 + C*(1 + 2*order)):

* materialized model row: (mu_x, mu_y, l11, l21, l22, rho, a[C], wx[C], wy[C])
* raw (optimized) row:    (mu_x, mu_y, s1,  l21, s2,  rho, a[C], wx[C], wy[C])

with L = [[l11, 0], [l21, l22]] the Cholesky factor of the covariance
(Sec. VI-B), s1 = ln l11, s2 = ln l22 (log-diagonal), rho = ln pi the mixing
weight (Eq. 4), a the expert constant and (wx, wy) the expert slope of a
linear ("steered") expert m(x) = a + W (x - mu).  order 0 = constant expert,
order 1 = linear expert.  Coordinates are in pixels, x = column, y = row,
pixel (c, r) has its centre at (c + 0.5, r + 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "num_params", "voronoi_ramps", "config1_image", "config2_image",
    "config3_images", "config5_images", "grid_init", "random_model",
    "fd_crop_case", "Workload", "SEEDS", "serving_models", "serving_requests",
    "batched_fit_inits",
]

SEEDS = {1: 1, 2: 2, 3: 3, 4: 4, 5: 5}


def num_params(C: int, order: int) -> int:
    """Floats per kernel row: mu(2) + Cholesky(3) + rho(1) + expert."""
    return 6 + C * (1 + 2 * order)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def voronoi_ramps(H: int, W: int, C: int, n_cells: int, rng: np.random.Generator,
                  slope: float = 0.005, base=(0.2, 0.8)) -> np.ndarray:
    """Piecewise-linear image: nearest-seed Voronoi cells, one ramp per cell.

    Per cell and channel: base ~ U(base), slope vector ~ U(-slope, slope)^2
    per pixel, measured from the cell's seed.  Returns float64 [H, W, C],
    unclipped.
    """
    from scipy.spatial import cKDTree

    seeds = rng.uniform(0.0, 1.0, size=(n_cells, 2)) * np.array([W, H], dtype=np.float64)
    b = rng.uniform(base[0], base[1], size=(n_cells, C))
    sl = rng.uniform(-slope, slope, size=(n_cells, C, 2))
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    xs += 0.5
    ys += 0.5
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1)
    _, idx = cKDTree(seeds).query(pts, k=1)
    idx = idx.reshape(H, W)
    dx = xs - seeds[idx, 0]
    dy = ys - seeds[idx, 1]
    img = b[idx] + sl[idx, :, 0] * dx[..., None] + sl[idx, :, 1] * dy[..., None]
    return img


def config1_image(seed: int = SEEDS[1], H: int = 64, W: int = 64, C: int = 1,
                  n_cells: int = 6, noise_var: float = 0.01) -> np.ndarray:
    """64x64 grey image: 6 Voronoi ramp cells + N(0, 0.01) noise, clipped.

    The noise figure is read as a variance (std 0.1), the convention the
    paper uses for its noise levels (Tables III/IV).
    """
    rng = _rng(seed)
    img = voronoi_ramps(H, W, C, n_cells, rng)
    img = img + rng.normal(0.0, math.sqrt(noise_var), size=img.shape)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def config2_image(seed: int = SEEDS[2], H: int = 512, W: int = 512, n_edges: int = 40) -> np.ndarray:
    """512x512 RGB: 40 local anisotropic step edges + sigma-3 texture + gradient."""
    from scipy.ndimage import gaussian_filter

    rng = _rng(seed)
    C = 3
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    xs += 0.5
    ys += 0.5
    c0 = rng.uniform(0.3, 0.7, size=C)
    cx = rng.uniform(-0.2, 0.2, size=C)
    cy = rng.uniform(-0.2, 0.2, size=C)
    img = c0 + cx * (xs / W)[..., None] + cy * (ys / H)[..., None]
    for _ in range(n_edges):
        px, py = rng.uniform(0, W), rng.uniform(0, H)
        th = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(32, 128)
        contrast = rng.uniform(0.2, 0.8) * (1 if rng.uniform() < 0.5 else -1)
        colour = rng.uniform(0.5, 1.0, size=C)
        d = (xs - px) * math.cos(th) + (ys - py) * math.sin(th)
        step = 1.0 / (1.0 + np.exp(-d))                     # 1 px logistic profile
        r = np.hypot(xs - px, ys - py)
        disc = 1.0 / (1.0 + np.exp(np.clip(r - rad, -60, 60)))  # soft disc window
        img += (contrast * (step - 0.5) * disc)[..., None] * colour
    tex = rng.normal(0.0, 1.0, size=(H, W, C))
    for c in range(C):
        tex[..., c] = gaussian_filter(tex[..., c], sigma=3.0, mode="wrap")
    tex /= tex.std()
    img += 0.1 * tex
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def step_edge_image(seed: int = 21, H: int = 256, W: int = 256, C: int = 1, n_lines: int = 6,
                    noise_std: float = 0.0) -> np.ndarray:
    """Piecewise-constant image with sharp edges (the 2D counterpart of the 1D step signal of
    Fig. 2): n_lines random straight lines cut the image into cells, each cell a constant
    colour in [0.1, 0.9]; the edges are exact pixel-centre steps.  Optional Gaussian noise."""
    rng = _rng(seed)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    xs += 0.5
    ys += 0.5
    code = np.zeros((H, W), dtype=np.int64)
    for k in range(n_lines):
        px, py = rng.uniform(0, W), rng.uniform(0, H)
        th = rng.uniform(0, math.pi)
        side = (xs - px) * math.cos(th) + (ys - py) * math.sin(th) > 0
        code |= side.astype(np.int64) << k
    levels = rng.uniform(0.1, 0.9, size=(1 << n_lines, C))
    img = levels[code]
    if noise_std > 0:
        img = img + rng.normal(0.0, noise_std, size=img.shape)
    return img.astype(np.float32)


def config3_images(seed: int = SEEDS[3], H: int = 2048, W: int = 2048,
                   noise_std: float = 25.0 / 255.0):
    """Denoising workload: (clean, noisy target), float32 [H, W, 3].

    Clean = the Voronoi-ramp generator scaled to keep its per-pixel
    statistics (6 cells per 64x64 area), clipped; target = clean +
    N(0, (25/255)^2), not clipped.
    """
    rng = _rng(seed)
    n_cells = max(1, int(round(6.0 * H * W / (64.0 * 64.0))))
    clean = np.clip(voronoi_ramps(H, W, 3, n_cells, rng), 0.0, 1.0)
    noisy = clean + rng.normal(0.0, noise_std, size=clean.shape)
    return clean.astype(np.float32), noisy.astype(np.float32)


def config5_images(seed: int = SEEDS[5], n: int = 64, lo: int = 128, hi: int = 1024):
    """Batched-fit workload: n RGB images with log-uniform sides (multiples of 8)."""
    rng = _rng(seed)
    out = []
    for _ in range(n):
        w = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 8.0)) * 8
        h = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 8.0)) * 8
        cells = max(1, int(round(6.0 * h * w / 4096.0)))
        img = voronoi_ramps(h, w, 3, cells, rng)
        img = img + rng.normal(0.0, 0.1, size=img.shape)
        out.append(np.clip(img, 0.0, 1.0).astype(np.float32))
    return out


def grid_init(image: np.ndarray, gx: int, gy: int, sigma: float = 4.0, order: int = 0):
    """Kernels on a gx x gy grid, round, unit mixing weight, expert = image at centre.

    Centres ((i + 0.5) W / gx, (j + 0.5) H / gy), kernel id j * gx + i.
    l11 = l22 = sigma, l21 = 0, rho = 0, a = image[floor(mu_y), floor(mu_x)],
    slopes 0.  Returns (raw, model), both float32 [K, NP]: the raw row holds
    s = float32(ln sigma), the model row holds l = sigma exactly.
    """
    H, W, C = image.shape
    K = gx * gy
    NP = num_params(C, order)
    raw = np.zeros((K, NP), dtype=np.float32)
    j, i = np.mgrid[0:gy, 0:gx]
    mux = ((i.ravel() + 0.5) * (W / gx)).astype(np.float32)
    muy = ((j.ravel() + 0.5) * (H / gy)).astype(np.float32)
    raw[:, 0] = mux
    raw[:, 1] = muy
    raw[:, 2] = np.float32(math.log(sigma))
    raw[:, 4] = np.float32(math.log(sigma))
    a = image[np.floor(muy).astype(int), np.floor(mux).astype(int), :]
    raw[:, 6:6 + C] = a
    model = raw.copy()
    model[:, 2] = np.float32(sigma)
    model[:, 4] = np.float32(sigma)
    return raw, model


def random_init(image: np.ndarray, K: int, sigma: float = 5.0, seed: int = 0, order: int = 0):
    """K round kernels at uniformly random centres with a fixed standard deviation (the
    random initialisation with a fixed scaling of 5 pixels, Sec. VI-B), unit mixing weight,
    expert constant = the image at the centre, zero slopes.  Returns the raw rows float32
    [K, NP] (log-diagonal Cholesky)."""
    rng = _rng(seed + 11)
    H, W, C = image.shape
    raw = np.zeros((K, num_params(C, order)), dtype=np.float32)
    raw[:, 0] = rng.uniform(0.0, W, K)
    raw[:, 1] = rng.uniform(0.0, H, K)
    raw[:, 2] = raw[:, 4] = np.float32(math.log(sigma))
    raw[:, 6:6 + C] = image[np.floor(raw[:, 1]).astype(int), np.floor(raw[:, 0]).astype(int), :]
    return raw


def random_model(K: int, C: int, order: int, W: int, H: int, seed: int,
                 sig_lo: float = 1.0, sig_hi: float = 10.0, margin: float = 12.0,
                 shear: float = 0.6, rho_std: float = 0.5, slope_std: float = 0.02):
    """Random materialized model with anisotropic, rotated kernels.

    Centres are uniform over the image enlarged by `margin` pixels on every
    side, so some kernels are clipped by or lie fully outside the raster.
    Returns float32 [K, NP] in the materialized layout.
    """
    rng = _rng(seed)
    NP = num_params(C, order)
    m = np.zeros((K, NP), dtype=np.float64)
    m[:, 0] = rng.uniform(-margin, W + margin, size=K)
    m[:, 1] = rng.uniform(-margin, H + margin, size=K)
    m[:, 2] = np.exp(rng.uniform(math.log(sig_lo), math.log(sig_hi), size=K))
    m[:, 4] = np.exp(rng.uniform(math.log(sig_lo), math.log(sig_hi), size=K))
    m[:, 3] = rng.uniform(-shear, shear, size=K) * np.minimum(m[:, 2], m[:, 4]) * 2.0
    m[:, 5] = rng.normal(0.0, rho_std, size=K)
    m[:, 6:6 + C] = rng.uniform(0.0, 1.0, size=(K, C))
    if order == 1:
        m[:, 6 + C:6 + 3 * C] = rng.normal(0.0, slope_std, size=(K, 2 * C))
    return m.astype(np.float32)


def stretched_model(K: int, C: int, order: int, W: int, H: int, seed: int,
                    size_lo: float = 0.5, size_hi: float = 9.0, max_aspect: float = 8.0):
    """Random materialized model whose kernels are ellipses of major standard deviation a in
    [size_lo, size_hi], aspect ratio up to max_aspect, at uniform angles (the shapes a long
    fit produces).  L is the Cholesky factor of R diag(a^2, b^2) R^T.  Float32 [K, NP]."""
    rng = _rng(seed + 7)
    m = random_model(K, C, order, W, H, seed).astype(np.float64)
    th = rng.uniform(0.0, np.pi, K)
    a = rng.uniform(size_lo, size_hi, K)
    b = a / rng.uniform(1.0, max_aspect, K)
    c, sn = np.cos(th), np.sin(th)
    sxx = (c * a) ** 2 + (sn * b) ** 2
    sxy = c * sn * (a * a - b * b)
    syy = (sn * a) ** 2 + (c * b) ** 2
    l11 = np.sqrt(sxx)
    l21 = sxy / l11
    m[:, 2], m[:, 3], m[:, 4] = l11, l21, np.sqrt(syy - l21 ** 2)
    return m.astype(np.float32)


def fd_crop_case(seed: int = SEEDS[3], size: int = 32, g: int = 4, order: int = 1):
    """Small gradient-check case: a size^2 RGB crop of the denoising target,
    K = g*g linear kernels from the grid init, randomly perturbed so every
    parameter's path is exercised.  Returns (target f32 [size,size,3],
    raw f32 [K,NP]) with raw in the raw layout."""
    rng = _rng(seed + 1000)
    clean, noisy = config3_images(seed, H=128, W=128)
    y0, x0 = 40, 56
    tgt = noisy[y0:y0 + size, x0:x0 + size, :].copy()
    raw, _ = grid_init(tgt, g, g, sigma=4.0, order=order)
    K = raw.shape[0]
    C = 3
    raw = raw.astype(np.float64)
    raw[:, 0:2] += rng.uniform(-1.5, 1.5, size=(K, 2))
    raw[:, 2] += rng.uniform(-0.25, 0.25, size=K)
    raw[:, 4] += rng.uniform(-0.25, 0.25, size=K)
    raw[:, 3] = rng.uniform(-1.0, 1.0, size=K)
    raw[:, 5] = rng.uniform(-0.5, 0.5, size=K)
    raw[:, 6:6 + C] += rng.uniform(-0.1, 0.1, size=(K, C))
    if order == 1:
        raw[:, 6 + C:6 + 3 * C] = rng.uniform(-0.03, 0.03, size=(K, 2 * C))
    return tgt, raw.astype(np.float32)


SERVING_KS = (256, 1024, 4096, 16384, 65536)


def serving_models(seed: int = SEEDS[4], n: int = 16, small: bool = False):
    """The resident models of the serving workload, as fit inputs: n RGB images and their
    grid initialisations with linear experts.  Model i has K = SERVING_KS[i % 5] kernels
    and a square native raster of side clip(sqrt(64 K), 256, 2048) (one kernel per 8x8
    pixels, as the batched fit), or a quarter of that side with small=True.  Returns a
    list of dicts (image f32 [H, W, 3], raw0 f32 [K, NP], K, side)."""
    rng = _rng(seed)
    out = []
    for i in range(n):
        K = SERVING_KS[i % len(SERVING_KS)]
        side = int(min(2048, max(256, round(math.sqrt(64.0 * K)))))
        g = int(round(math.sqrt(K)))
        if small:
            side //= 4
            g = max(2, g // 4)
        cells = max(1, int(round(6.0 * side * side / 4096.0)))
        img = voronoi_ramps(side, side, 3, cells, rng)
        img = np.clip(img + rng.normal(0.0, 0.01, size=img.shape), 0.0, 1.0).astype(np.float32)
        raw, _ = grid_init(img, g, g, sigma=0.5 * side / g, order=1)
        out.append(dict(image=img, raw0=raw, K=g * g, side=side))
    return out


def serving_requests(sides, n: int, rate: float = 200.0, seed: int = SEEDS[4] + 100,
                     scales=(1, 2, 3, 4), max_side: int = 4096, poisson: bool = True):
    """A render request stream over resident models with native sides `sides`.

    Each request picks a model uniformly, an upscale factor uniformly from `scales`, and
    an output window of min(max_side, side * scale) pixels per axis at a uniform origin
    inside the upscaled raster.  Arrival times (seconds) are a Poisson process of the
    given rate (exponential gaps), or all zero with poisson=False.  Returns a list of
    dicts (model, scale, width, height, origin_x, origin_y, arrival)."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        m = int(rng.integers(len(sides)))
        s = int(scales[int(rng.integers(len(scales)))])
        full = sides[m] * s
        w = h = min(max_side, full)
        ox = int(rng.integers(full - w + 1))
        oy = int(rng.integers(full - h + 1))
        if poisson:
            t += float(rng.exponential(1.0 / rate))
        out.append(dict(model=m, scale=s, width=w, height=h, origin_x=ox, origin_y=oy,
                        arrival=t if poisson else 0.0))
    return out


def batched_fit_inits(images, order: int = 1):
    """Grid initialisations for a batch of images, one kernel per 8x8 pixels
    (K = H W / 64, grid W/8 x H/8, sigma 4 px)."""
    out = []
    for img in images:
        H, W, _ = img.shape
        raw, _ = grid_init(img, max(1, W // 8), max(1, H // 8), sigma=4.0, order=order)
        out.append(raw)
    return out


@dataclass
class Workload:
    """A fit workload: target image, initial raw parameters and fit settings."""
    name: str
    target: np.ndarray          # float32 [H, W, C]
    raw0: np.ndarray            # float32 [K, NP] raw layout
    order: int
    steps: int
    clean: np.ndarray | None = None

    @property
    def K(self) -> int:
        return self.raw0.shape[0]


def workload(n: int, small: bool = False) -> Workload:
    """The fit workloads by number: 1 (64^2 grey, K=64 const), 2 (512^2 RGB,
    K=4096 linear), 3 (2048^2 RGB denoising, K=65536 linear)."""
    if n == 1:
        img = config1_image()
        raw, _ = grid_init(img, 8, 8, 4.0, order=0)
        return Workload("fit-64x64-grey-K64-const", img, raw, 0, 100)
    if n == 2:
        img = config2_image()
        raw, _ = grid_init(img, 64, 64, 4.0, order=1)
        return Workload("fit-512x512-rgb-K4096-linear", img, raw, 1, 2000)
    if n == 3:
        clean, noisy = config3_images()
        raw, _ = grid_init(noisy, 256, 256, 4.0, order=1)
        return Workload("fit-2048x2048-rgb-K65536-linear-denoise", noisy, raw, 1, 1000,
                        clean=clean)
    raise ValueError(f"no fit workload {n}")
