"""Device-memory plumbing around the C ABI: workspaces, fit state, convenience calls.

PyTorch provides device memory (tensors from its caching allocator) and the
current HIP stream; every computation is a call into ``libsmoe.so``.
"""
from __future__ import annotations

import ctypes as ct
import math
from dataclasses import dataclass

import torch

from . import _capi as C

TILE = C.TILE


def num_params(C_: int, order: int) -> int:
    """Floats per kernel row: mu(2) + Cholesky(3) + rho(1) + expert."""
    return 6 + C_ * (1 + 2 * order)


def tiles(width: int, height: int, origin_x: int = 0, origin_y: int = 0) -> int:
    """Blocks of a raster: the 16x16 blocks of its scale's output grid, aligned to multiples of
    16 in the output coordinate, that its pixels touch."""
    def across(n, o):
        return (o + n - 1) // TILE - o // TILE + 1
    return across(width, origin_x) * across(height, origin_y)


BOXES = {"square": C.SMOE_BOX_SQUARE, "tight": C.SMOE_BOX_TIGHT}


def _box(box) -> int:
    b = BOXES.get(box, box)
    if b not in BOXES.values():
        raise ValueError(f"box must be one of {sorted(BOXES)}")
    return b


MODES = {"smoe": C.SMOE_MODE_SMOE, "rbf": C.SMOE_MODE_RBF}


def _mode(mode) -> int:
    m = MODES.get(mode, mode)
    if m not in MODES.values():
        raise ValueError(f"mode must be one of {sorted(MODES)}")
    return m


TRUNCS = {"render": C.SMOE_TRUNC_RENDER, "gradient": C.SMOE_TRUNC_GRADIENT}


def _trunc(trunc) -> int:
    t = TRUNCS.get(trunc, trunc)
    if t not in TRUNCS.values():
        raise ValueError(f"trunc must be one of {sorted(TRUNCS)}")
    return t


def make_grid(width, height, scale=1, origin_x=0, origin_y=0, radius=3.0,
              sharpen=1.0, box="square", mode="smoe", trunc="gradient") -> C.SmoeGrid:
    """Output raster; sharpen = f renders every kernel with its bandwidth divided by f
    (native sharpening by kernel editing, Sec. II-B), 1 = none.  box: "square" (the
    square box of Sec. IV-B) or "tight" (the ellipse's axis-aligned extents: the same
    image from shorter block lists).  mode: "smoe" (the gated regression, Eq. 2-4) or
    "rbf" (the un-normalised weighted sum of kernels, Eq. 1).  trunc: where the ellipse test
    applies -- "gradient" (the render takes every kernel of the block list; out-of-ellipse
    pixels are discarded in the gradient only, Sec. IV-B) or "render" (render and
    gradient)."""
    return C.SmoeGrid(int(width), int(height), int(scale), int(origin_x), int(origin_y),
                      float(radius), float(sharpen), _box(box), _mode(mode), _trunc(trunc))


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_params(params, C_, order):
    NP = num_params(C_, order)
    if not (params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()
            and params.dim() == 2 and params.shape[1] == NP):
        raise ValueError(f"params must be a contiguous cuda float32 [K, {NP}] tensor")


def model_struct(params: torch.Tensor, C_: int, order: int) -> C.SmoeModel:
    _check_params(params, C_, order)
    return C.SmoeModel(params.shape[0], C_, order, params.data_ptr())


class Bins:
    """A binning workspace (block lists, records, backward scratch) in one device buffer."""

    def __init__(self, K: int, C_: int, order: int, max_tiles: int, capacity: int,
                 device="cuda", render_only: bool = False, zero: bool = True):
        """render_only: no per-pair gradient scratch (bin + render only).  zero=False leaves
        the buffer uninitialised, which the binning and render calls allow (they write
        every word they read)."""
        self.K, self.C, self.order = K, C_, order
        self.max_tiles, self.capacity = int(max_tiles), int(capacity)
        size = C.smoe_render_workspace_bytes if render_only else C.smoe_bins_workspace_bytes
        n = size(K, C_, order, self.max_tiles, self.capacity)
        if n == 0:
            raise ValueError("invalid workspace shape")
        self.nbytes = n
        self.ws = (torch.zeros if zero else torch.empty)(n, dtype=torch.uint8, device=device)
        self.c = C.SmoeBins()
        lay = C.smoe_render_workspace_layout if render_only else C.smoe_bins_layout
        lay(self.c, self.ws.data_ptr(), n, K, C_, order, self.max_tiles, self.capacity)

    def _view(self, ptr: int, count: int, dtype) -> torch.Tensor:
        off = ptr - self.ws.data_ptr()
        size = torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + count * size].view(dtype)

    def tile_rects(self):
        return self._view(self.c.tile_rects, 4 * self.K, torch.int32).view(self.K, 4)

    def native_rects(self):
        return self._view(self.c.native_rects, 4 * self.K, torch.int32).view(self.K, 4)

    def counts(self):
        return self._view(self.c.counts, self.K, torch.int32)

    def ranges(self, T: int):
        return self._view(self.c.ranges, 2 * T, torch.int32).view(T, 2)

    def keys(self, P: int):
        return self._view(self.c.keys, P, torch.int32)

    def vals(self, P: int):
        return self._view(self.c.vals, P, torch.int32)

    def read_status(self, stream=None):
        """Synchronises the stream; returns (overflowed, [P needed, overflow, longest,
        non-finite]): the last word is 1 when a kernel row with a NaN or infinite parameter
        was met (it then takes part nowhere)."""
        code, st = C.smoe_read_status(self.c, _stream(stream))
        return code == C.SMOE_ERR_CAPACITY, st


def initial_capacity(K: int, T: int) -> int:
    return max(1024, 8 * K + 2 * T)


def bin(params: torch.Tensor, C_: int, order: int, grid: C.SmoeGrid, bins: Bins | None = None,
        capacity: int | None = None, stream=None, grow: bool = True) -> Bins:
    """smoe_bin; with grow=True the workspace is re-made until the pairs fit (host sync)."""
    m = model_struct(params, C_, order)
    T = tiles(grid.width, grid.height, grid.origin_x, grid.origin_y)
    if bins is None:
        bins = Bins(m.K, C_, order, T, capacity or initial_capacity(m.K, T), params.device)
    C.smoe_bin(m, grid, bins.c, _stream(stream))
    if grow:
        over, st = bins.read_status(stream)
        if over:
            bins = Bins(m.K, C_, order, max(T, bins.max_tiles), int(st[0] * 1.25) + 1024,
                        params.device)
            C.smoe_bin(m, grid, bins.c, _stream(stream))
    return bins


def render(params: torch.Tensor, C_: int, order: int, grid: C.SmoeGrid, bins: Bins | None = None,
           target: torch.Tensor | None = None, stream=None):
    """Bins (if not given) and renders.  Returns (image [H, W, C], denom [H, W], loss or
    None, bins)."""
    if bins is None:
        bins = bin(params, C_, order, grid, stream=stream)
    m = model_struct(params, C_, order)
    dev = params.device
    image = torch.empty((grid.height, grid.width, C_), dtype=torch.float32, device=dev)
    denom = torch.empty((grid.height, grid.width), dtype=torch.float32, device=dev)
    loss = None
    if target is not None:
        if not (target.is_cuda and target.dtype == torch.float32 and target.is_contiguous()
                and tuple(target.shape) == (grid.height, grid.width, C_)):
            raise ValueError("target must be a contiguous cuda float32 [H, W, C] tensor")
        loss = torch.empty((1,), dtype=torch.float32, device=dev)
    C.smoe_render(m, grid, bins.c, image.data_ptr(), denom.data_ptr(), _ptr(target), _ptr(loss),
                  _stream(stream))
    return image, denom, loss, bins


def render_noalloc(params: torch.Tensor, C_: int, order: int, grid: C.SmoeGrid, image=None,
                   denom=None, status=None, stream=None):
    """Bin + render through smoe_render_noalloc (the library's static workspace: no device
    allocation inside the call).  image [H, W, C], denom [H, W] and status int32[4] may be
    given preallocated (a caller that must not allocate passes all three); missing ones are
    allocated here, outside the library call.  Returns (image, denom, status)."""
    m = model_struct(params, C_, order)
    dev = params.device
    if image is None:
        image = torch.empty((grid.height, grid.width, C_), dtype=torch.float32, device=dev)
    if denom is None:
        denom = torch.empty((grid.height, grid.width), dtype=torch.float32, device=dev)
    if status is None:
        status = torch.empty(4, dtype=torch.int32, device=dev)
    for t, shape, dt in ((image, (grid.height, grid.width, C_), torch.float32),
                         (denom, (grid.height, grid.width), torch.float32),
                         (status, (4,), torch.int32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"output must be a contiguous cuda {dt} {shape} tensor")
    C.smoe_render_noalloc(m, grid, image.data_ptr(), denom.data_ptr(), status.data_ptr(),
                          _stream(stream))
    return image, denom, status


def render_backward(params, C_, order, grid, bins: Bins, image, denom, grad_image=None,
                    target=None, stream=None) -> torch.Tensor:
    """dL/dparams [K, NP] in raw order (mu, s1, l21, s2, rho, a, wx, wy)."""
    m = model_struct(params, C_, order)
    grads = torch.empty_like(params)
    for t in (image, denom, grad_image, target):
        if t is not None and not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("image/denom/grad_image/target must be contiguous cuda float32")
    C.smoe_render_backward(m, grid, bins.c, image.data_ptr(), denom.data_ptr(), _ptr(grad_image),
                           _ptr(target), grads.data_ptr(), _stream(stream))
    return grads


def materialize(raw: torch.Tensor, C_: int, order: int, stream=None) -> torch.Tensor:
    _check_params(raw, C_, order)
    out = torch.empty_like(raw)
    C.smoe_materialize(raw.shape[0], C_, order, raw.data_ptr(), out.data_ptr(), _stream(stream))
    return out


class Segments:
    """A laid-out segment table (host ctypes array + device copy) for batched calls.

    rasters: list of dicts with width, height and optionally scale, origin_x, origin_y,
    sharpen (1 = none), num_kernels, param_offset (default: the running sum of
    num_kernels)."""

    def __init__(self, rasters, device="cuda", stream=None):
        n = len(rasters)
        if n < 1:
            raise ValueError("at least one raster")
        self.host = (C.SmoeSegment * n)()
        k = 0
        for i, r in enumerate(rasters):
            sg = self.host[i]
            sg.width, sg.height = int(r["width"]), int(r["height"])
            sg.scale = int(r.get("scale", 1))
            sg.origin_x, sg.origin_y = int(r.get("origin_x", 0)), int(r.get("origin_y", 0))
            sg.sharpen = float(r.get("sharpen", 1.0))
            sg.num_kernels = int(r.get("num_kernels", 0))
            sg.param_offset = int(r.get("param_offset", k))
            k += sg.num_kernels
        self.K, self.T, self.pixels = C.smoe_segments_layout(self.host)
        # device copy: staged through pinned memory and copied on `stream` (no host wait)
        nbytes = ct.sizeof(self.host)
        pinned = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        ct.memmove(pinned.data_ptr(), ct.addressof(self.host), nbytes)
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            self.dev = pinned.to(device, non_blocking=True)
        self.n = n

    def __len__(self):
        return self.n

    def pixel_slices(self):
        """(start, stop, height, width) of every raster in the concatenated images."""
        return [(sg.pixel_offset, sg.pixel_offset + sg.width * sg.height, sg.height, sg.width)
                for sg in self.host]


def bin_batched(params: torch.Tensor, C_: int, order: int, segs: Segments, radius: float = 3.0,
                bins: Bins | None = None, capacity: int | None = None, stream=None,
                grow: bool = True, box="square", mode="smoe", trunc="gradient") -> Bins:
    """smoe_bin_batched over every segment; with grow=True the workspace is re-made until the
    pairs fit (host sync)."""
    _check_params(params, C_, order)
    batch = C.SmoeBatch(C_, order, params.data_ptr(), params.shape[0], segs.n, segs.dev.data_ptr(),
                        ct.addressof(segs.host), float(radius), _box(box), _mode(mode),
                        _trunc(trunc))
    if bins is None:
        bins = Bins(segs.K, C_, order, segs.T, capacity or initial_capacity(segs.K, segs.T),
                    params.device)
    C.smoe_bin_batched(batch, bins.c, _stream(stream))
    if grow:
        over, st = bins.read_status(stream)
        if over:
            bins = Bins(segs.K, C_, order, max(segs.T, bins.max_tiles), int(st[0] * 1.25) + 1024,
                        params.device)
            C.smoe_bin_batched(batch, bins.c, _stream(stream))
    return bins


def render_batched(params: torch.Tensor, C_: int, order: int, segs: Segments, bins: Bins,
                   images: torch.Tensor, denoms: torch.Tensor | None = None, radius: float = 3.0,
                   stream=None, box="square", mode="smoe", trunc="gradient"):
    """smoe_render_batched into the concatenated images [total pixels, C]."""
    _check_params(params, C_, order)
    batch = C.SmoeBatch(C_, order, params.data_ptr(), params.shape[0], segs.n, segs.dev.data_ptr(),
                        ct.addressof(segs.host), float(radius), _box(box), _mode(mode),
                        _trunc(trunc))
    C.smoe_render_batched(batch, bins.c, images.data_ptr(), _ptr(denoms), _stream(stream))
    return images


def fuse_windows(window_images: torch.Tensor, C_: int, width: int, height: int,
                 displacement: int, window: int = 16, out: torch.Tensor | None = None,
                 stream=None) -> torch.Tensor:
    """smoe_fuse_windows: the mean over the covering windows (Sec. V-C, Eq. (11)) of the
    window renders [m^2 width height, C] (window order, as smoe_fuse_windows documents)
    into out [height, width, C]."""
    m = window // displacement if displacement > 0 else 0
    if not (window_images.is_cuda and window_images.dtype == torch.float32
            and window_images.is_contiguous()):
        raise ValueError("window_images must be a contiguous cuda float32 tensor")
    if window_images.numel() != m * m * width * height * C_:
        raise ValueError("window_images must hold (window/displacement)^2 * width * height * C "
                         "floats")
    if out is None:
        out = torch.empty((height, width, C_), dtype=torch.float32, device=window_images.device)
    C.smoe_fuse_windows(window_images.data_ptr(), C_, width, height, window, displacement,
                        out.data_ptr(), _stream(stream))
    return out


@dataclass
class AdamConfig:
    """Adam settings (Sec. VI-B): centre rate decays exponentially to lr_mu_final."""
    lr_mu: float = 1e-2
    lr_mu_final: float = 1e-5
    lr_chol: float = 1e-3
    lr_rho: float = 1e-3
    lr_expert: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    total_steps: int = 10000

    @classmethod
    def constant(cls, lr: float, total_steps: int = 1):
        return cls(lr, lr, lr, lr, lr, total_steps=total_steps)

    def c(self) -> C.SmoeAdamConfig:
        return C.SmoeAdamConfig(self.lr_mu, self.lr_mu_final, self.lr_chol, self.lr_rho,
                                self.lr_expert, self.beta1, self.beta2, self.eps,
                                int(self.total_steps))


class FitState:
    """Device state of one fit, driven by smoe_fit_step (one call = one iteration).

    target: one cuda float32 [H, W, C] image with raw0 [K, NP] -- or, for a batched fit, a
    list of images with a list of raw0 arrays (one per image): the images are fitted together
    in lock-step, each by its own kernels, with one launch per stage for all of them.
    radius, box, mode, trunc: the rule's settings, as in make_grid (mode "rbf" fits the
    weighted sum of kernels of Eq. 1).  write_render: whether each step stores its render in
    `image` / `denom` (set_write_render changes it; a graph captures the value it had)."""

    def __init__(self, target, raw0, order: int, adam: AdamConfig, max_steps: int = 0,
                 capacity: int | None = None, radius: float = 3.0, box="square",
                 mode="smoe", trunc="gradient", write_render: bool = True):
        self.write_render = bool(write_render)
        batched = isinstance(target, (list, tuple))
        targets = list(target) if batched else [target]
        raws = list(raw0) if batched else [raw0]
        if len(targets) != len(raws) or not targets:
            raise ValueError("one raw parameter array per target image")
        for t in targets:
            if not (t.dtype == torch.float32 and t.dim() == 3 and (batched or t.is_cuda)):
                raise ValueError("targets must be float32 [H, W, C] tensors (cuda unless "
                                 "several images are fitted together)")
        C_ = targets[0].shape[2]
        # a batch may come from host memory: it is concatenated there and moved once
        dev = targets[0].device if targets[0].is_cuda else torch.device("cuda")
        self.C, self.order, self.batched = C_, order, batched
        self.shapes = [tuple(t.shape[:2]) for t in targets]
        self.raw = torch.cat([r.to(dtype=torch.float32) for r in raws]).to(dev).contiguous()
        _check_params(self.raw, C_, order)
        self.K = self.raw.shape[0]
        self.segments = None
        if batched:
            self.segments = Segments([{"width": w, "height": h, "num_kernels": r.shape[0]}
                                      for (h, w), r in zip(self.shapes, raws)], device=dev)
            self.target = torch.cat([t.reshape(-1, C_) for t in targets]).to(dev).contiguous()
            npx = self.target.shape[0]
            self.image = torch.zeros((npx, C_), dtype=torch.float32, device=dev)
            self.denom = torch.zeros((npx,), dtype=torch.float32, device=dev)
            T = self.segments.T
            self.H = self.W = None
        else:
            self.target = targets[0].contiguous()
            H, W = self.shapes[0]
            self.H, self.W = H, W
            self.image = torch.zeros((H, W, C_), dtype=torch.float32, device=dev)
            self.denom = torch.zeros((H, W), dtype=torch.float32, device=dev)
            T = tiles(W, H)
        self.m = torch.zeros_like(self.raw)
        self.v = torch.zeros_like(self.raw)
        self.model = materialize(self.raw, C_, order)
        self.grads = torch.zeros_like(self.raw)
        self.max_steps = int(max_steps)
        self.loss_history = torch.zeros(max(1, self.max_steps), dtype=torch.float32, device=dev)
        self.step_counter = torch.zeros(1, dtype=torch.int32, device=dev)
        self.scalars = torch.zeros(4, dtype=torch.float32, device=dev)
        H0, W0 = self.shapes[0]
        self.grid = make_grid(W0, H0, 1, 0, 0, radius, box=box, mode=mode, trunc=trunc)
        self.box, self.mode, self.trunc = box, mode, trunc
        self.adam = adam
        if capacity is None:
            if batched:
                b = bin_batched(self.model, C_, order, self.segments, radius, box=box)
            else:
                b = bin(self.model, C_, order, self.grid)
            _, st = b.read_status()
            # the fit step's buckets: room for twice the initial longest list (at least 64)
            capacity = T * max(64, 2 * int(st[2]))
        self.bins = Bins(self.K, C_, order, T, capacity, dev)
        self._build_struct()

    def _build_struct(self):
        seg = self.segments
        self.c = C.SmoeFitState(
            self.K, self.C, self.order, self.grid, self.adam.c(), self.raw.data_ptr(),
            self.m.data_ptr(), self.v.data_ptr(), self.model.data_ptr(), self.grads.data_ptr(),
            self.image.data_ptr(), self.denom.data_ptr(), self.loss_history.data_ptr(),
            self.max_steps, 0, 1 if self.write_render else 0, self.step_counter.data_ptr(),
            self.scalars.data_ptr(),
            0 if seg is None else seg.n, None if seg is None else seg.dev.data_ptr(),
            None if seg is None else ct.addressof(seg.host), self.bins.c)

    def set_write_render(self, on: bool):
        """Whether the following steps store their render in image / denom."""
        self.write_render = bool(on)
        self.c.write_render = 1 if on else 0

    def segment_losses(self, stream=None) -> torch.Tensor:
        """Each image's MSE at the last step (a single-image fit gives one value)."""
        n = 1 if self.segments is None else self.segments.n
        out = torch.zeros(n, dtype=torch.float32, device=self.raw.device)
        C.smoe_fit_segment_losses(self.c, out.data_ptr(), _stream(stream))
        return out

    def images(self):
        """The last step's render, one [H, W, C] view per image."""
        if self.segments is None:
            return [self.image]
        return [self.image[a:b].view(h, w, self.C) for a, b, h, w in self.segments.pixel_slices()]

    def raw_rows(self):
        """The raw parameter rows of each image."""
        if self.segments is None:
            return [self.raw]
        return [self.raw[sg.kernel_offset:sg.kernel_offset + sg.num_kernels]
                for sg in self.segments.host]

    def step(self, loss_out: torch.Tensor | None = None, stream=None):
        C.smoe_fit_step(self.c, self.target.data_ptr(), _ptr(loss_out), _stream(stream))

    def step_timed(self, events4, stream=None):
        """One step with hipEvent_t handles recorded at the stage boundaries (None = skip):
        start, after binning, after the per-block render+backward kernel, after Adam."""
        C.smoe_fit_step_timed(self.c, self.target.data_ptr(), None, events4, _stream(stream))

    def capture(self, steps: int, events=None) -> "torch.cuda.CUDAGraph":
        """Captures `steps` fit steps into one HIP graph (nothing runs during capture).
        Each replay advances the fit by `steps` (the step counter lives on the device).
        events: optional list of `steps` four-entry event lists for smoe_fit_step_timed.
        A re-made workspace (grow_if_needed) invalidates the graph."""
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        prepared = self.c.prepared  # capture runs nothing: the device state is unchanged
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                for i in range(steps):
                    if events is None:
                        self.step()
                    else:
                        self.step_timed(events[i])
        torch.cuda.current_stream().wait_stream(side)
        self.c.prepared = prepared
        return g

    def replay(self, graph: "torch.cuda.CUDAGraph"):
        """Replays a graph from capture(); afterwards the workspace is prepared."""
        graph.replay()
        self.c.prepared = 1

    def run_graphed(self, steps: int, steps_per_graph: int = 32, check_every: int = 4):
        """Like run(), replaying captured graphs of steps_per_graph steps; re-captures after
        a workspace re-size and finishes any remainder with eager steps."""
        goal = self.steps_done() + steps
        graph = None
        while True:
            todo = goal - self.steps_done()
            if todo <= 0:
                break
            if todo < steps_per_graph:
                for _ in range(todo):
                    self.step()
            else:
                if graph is None:
                    graph = self.capture(steps_per_graph)
                for _ in range(min(check_every, todo // steps_per_graph)):
                    self.replay(graph)
            if self.grow_if_needed():
                graph = None
        return self

    def steps_done(self) -> int:
        return int(self.step_counter.item())

    def grow_if_needed(self, stream=None) -> bool:
        """Host sync; after a pair-capacity overflow re-makes the workspace larger."""
        over, st = self.bins.read_status(stream)
        if over:
            # status[0]: blocks x the longest list the step met
            self.bins = Bins(self.K, self.C, self.order, self.bins.max_tiles,
                             max(int(st[0] * 1.5), self.bins.capacity + 1), self.raw.device)
            self._build_struct()
        return over

    def run(self, steps: int, check_every: int = 64, stream=None):
        """Runs until `steps` more iterations have completed, re-sizing on overflow."""
        goal = self.steps_done() + steps
        while True:
            todo = goal - self.steps_done()
            if todo <= 0:
                break
            for _ in range(min(todo, check_every)):
                self.step(stream=stream)
            self.grow_if_needed(stream)
        return self

    def losses(self) -> torch.Tensor:
        n = min(self.steps_done(), self.max_steps)
        return self.loss_history[:n]


def psnr(a: torch.Tensor, b: torch.Tensor, peak: float = 1.0) -> float:
    mse = torch.mean((a.double() - b.double()) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)
