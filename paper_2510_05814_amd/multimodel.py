"""Multi-model fusion for denoising (Sec. V-C, Eq. 10-14): block-overlapping SMoE models.

A 16x16 window is shifted over the image by a displacement d in both directions; for every
window position an SMoE model is fitted to the window's noisy pixels alone, and each pixel's
estimate is the average of the predictions of all windows that cover it (Eq. 10).  With
windows at offsets -(16 - d), -(16 - d) + d, ... every pixel is covered by (16 / d)^2
windows (windows that reach past the border are clipped to the image), so d = 16, 8, 4, 2
give H = 1, 4, 16, 64 hypotheses per pixel.

All windows are fitted together as one batched fit (each window is a segment of the
segment table, with its own kernels), one launch sequence per step for all of them; the
average of Eq. (11) is smoe_fuse_windows, a fixed-order gather over the window renders.
"""
from __future__ import annotations

import numpy as np
import torch

from .core import AdamConfig, FitState, bin_batched, fuse_windows, render_batched

WINDOW = 16


def window_layout(height: int, width: int, d: int, window: int = WINDOW):
    """Window rectangles (y0, x0, h, w), clipped to the image, for displacement d: offsets
    -(window - d) + k d along each axis, every pixel covered by (window / d)^2 windows."""
    if d < 1 or window % d:
        raise ValueError("the displacement must divide the window size")

    def axis(n):
        out = []
        for o in range(-(window - d), n, d):
            a, b = max(0, o), min(n, o + window)
            if b > a:
                out.append((a, b - a))
        return out

    return [(y0, x0, h, w) for (y0, h) in axis(height) for (x0, w) in axis(width)]


def _grid_init(crop: np.ndarray, spacing: int, sigma: float, order: int) -> np.ndarray:
    """Raw rows of a window: kernels on a grid of the given spacing (at least one), round,
    unit mixing weight, expert constant = the noisy pixel under the centre, zero slopes."""
    h, w, C = crop.shape
    gx, gy = max(1, round(w / spacing)), max(1, round(h / spacing))
    NP = 6 + C * (1 + 2 * order)
    j, i = np.mgrid[0:gy, 0:gx]
    mux = (i.ravel() + 0.5) * (w / gx)
    muy = (j.ravel() + 0.5) * (h / gy)
    raw = np.zeros((gx * gy, NP), np.float32)
    raw[:, 0], raw[:, 1] = mux, muy
    raw[:, 2] = raw[:, 4] = np.float32(np.log(sigma))
    raw[:, 6:6 + C] = crop[np.floor(muy).astype(int), np.floor(mux).astype(int), :]
    return raw


class MultiModelDenoiser:
    """Fits every window of displacement d to its noisy pixels and fuses the predictions."""

    def __init__(self, noisy: np.ndarray, d: int, spacing: int = 8, sigma: float = 4.0,
                 order: int = 1, adam: AdamConfig | None = None, max_steps: int = 0):
        noisy = np.ascontiguousarray(noisy, dtype=np.float32)
        self.H, self.W, self.C = noisy.shape
        self.d = d
        self.windows = window_layout(self.H, self.W, d)
        crops = [noisy[y0:y0 + h, x0:x0 + w] for (y0, x0, h, w) in self.windows]
        raws = [_grid_init(c, spacing, sigma, order) for c in crops]
        # host tensors: the batch is concatenated on the host and moved once
        tg = [torch.from_numpy(np.ascontiguousarray(c)) for c in crops]
        rw = [torch.from_numpy(r) for r in raws]
        # a window's block list holds at most the window's own kernels
        width = max(r.shape[0] for r in raws)
        blocks = sum(((h + 15) // 16) * ((w + 15) // 16) for (_, _, h, w) in self.windows)
        self.state = FitState(tg, rw, order, adam or AdamConfig(), max_steps=max_steps,
                              capacity=blocks * width)
    @property
    def hypotheses(self) -> int:
        return (WINDOW // self.d) ** 2

    def fit(self, steps: int, graphed: bool = True):
        if graphed:
            self.state.run_graphed(steps)
        else:
            self.state.run(steps)
        return self

    def window_images(self) -> torch.Tensor:
        """Every window's render of its current model, concatenated [pixels, C]."""
        st = self.state
        bins = bin_batched(st.model, self.C, st.order, st.segments)
        out = torch.empty((st.segments.pixels, self.C), dtype=torch.float32,
                          device=st.model.device)
        render_batched(st.model, self.C, st.order, st.segments, bins, out)
        return out

    def image(self) -> torch.Tensor:
        """The fused estimate [H, W, C] (Eq. 11): the mean over the windows covering each pixel
        of their current models' predictions."""
        return fuse_windows(self.window_images(), self.C, self.W, self.H, self.d, WINDOW)
