"""Serving render: fitted SMoE models kept resident in HBM and rendered on request.

A request names a resident model, an integer upscale factor s and an output window
(width, height, origin) in the upscaled raster.  Output pixel (u, v) samples the
continuous regression (Eq. 3-5) at native coordinate ((origin + u) + 0.5) / s, so every
factor is a native super-resolution of the same model, not an interpolation of a render.
A request may also ask for native sharpening by a factor f: every kernel is rendered with
its bandwidth divided by f (kernel editing, Sec. II-B), the resident model unchanged.

Two servers share the request format and the report:

* ``Server`` -- continuous batching.  Requests that have arrived wait in a FIFO queue.
  Whenever one of its streams is free, the batches in flight leave part of the GPU idle
  (fewer blocks than it renders at once) and, if a batch is in flight, a backlog has formed
  (at least two requests wait), the server takes the queue's head requests whose
  memory (output image + their share of the binning workspace) fits the HBM budget beside
  the batches still in flight, lays them out as segments of one raster table, and issues
  one batched binning and ONE render launch over the concatenated (request, block) list on
  that stream.  Batches on different streams overlap on the device; finished batches
  release their memory, stream and blocks, and the queue is admitted again.  Nothing waits
  on the device except to learn which batches have finished.
* ``PlainServer`` -- the baseline: one bin + render launch sequence per request, in
  arrival order on one stream, the host waiting for each request before the next.

Latency of a request = device completion time of its render - arrival time, both on the
host clock (the completion time is the request's completion event measured against a
reference event recorded at the start).  The workspace of a batch is sized from an upper
bound of its (block, kernel) pairs computed on the host from the resident models' box
sizes (Sec. IV-B), so no batch needs a host round-trip to learn its pair count.
"""
from __future__ import annotations

import contextlib
import ctypes as ct
import gc
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _capi as C
from .core import Bins, _box, _check_params, _mode, _trunc, make_grid, model_struct

TILE = 16


@dataclass
class RenderRequest:
    model: int
    scale: int
    width: int
    height: int
    origin_x: int = 0
    origin_y: int = 0
    arrival: float = 0.0      # seconds from the start of the run
    sharpen: float = 1.0      # bandwidth divisor f (1 = none)


@dataclass
class RenderResult:
    request: RenderRequest
    done: float               # device completion, seconds from the start of the run
    batch: int
    image: torch.Tensor | None = None
    started: float = 0.0      # device start of its batch's first launch, same clock

    @property
    def latency(self) -> float:
        return self.done - self.request.arrival


class BoxSpans:
    """Host-side upper bounds of the (block, kernel) pairs a render creates, from each
    kernel's square box (half-side r sqrt(lambda_max) of its covariance, Sec. IV-B): the
    native 16x16 blocks the box overlaps, and the output blocks holding a sample point in
    them.

    models: float64/float32 [K_i, NP] materialized rows, one array per model."""

    def __init__(self, models, radius: float = 3.0):
        self.radius = float(radius)
        self._R = []
        for m in models:
            m = np.asarray(m, dtype=np.float64)
            l11, l21, l22 = m[:, 2], m[:, 3], m[:, 4]
            sxx, sxy, syy = l11 * l11, l11 * l21, l21 * l21 + l22 * l22
            lam = 0.5 * (sxx + syy) + np.sqrt((0.5 * (sxx - syy)) ** 2 + sxy * sxy)
            self._R.append(self.radius * np.sqrt(lam))
        self._spans = {}

    def _span_table(self, i: int, scale: int, sharpen: float = 1.0):
        """Sorted per-kernel bound on the blocks its box spans per axis, with prefix sums."""
        f = 1.0 if sharpen in (0.0, 1.0) else float(sharpen)
        key = (i, scale, f)
        if key not in self._spans:
            # native blocks overlapped per axis: nb <= floor(2 R / (16 f)) + 2 (sharpening
            # divides L, hence R, by f; the 1e-5 absorbs the binary32 rounding of the box
            # edges); their sample points at scale s are 16 s nb consecutive output pixels
            # (points sit half a spacing off every block boundary), which touch at most
            # s nb + 1 output blocks.
            nb = np.floor(2.0 * self._R[i] / (TILE * f) * (1.0 + 1e-5)).astype(np.int64) + 2
            b = np.sort(nb * scale + 1)
            self._spans[key] = (b, np.concatenate([[0], np.cumsum(b)]),
                                np.concatenate([[0], np.cumsum(b * b)]))
        return self._spans[key]

    def pair_bound(self, i: int, scale: int, width: int, height: int,
                   sharpen: float = 1.0) -> int:
        """Sum over model i's kernels of min(span, blocks across) * min(span, blocks down),
        with the most blocks a window of this size touches at any origin."""
        b, s1, s2 = self._span_table(i, scale, sharpen)
        a = (width + TILE - 2) // TILE + 1
        c = (height + TILE - 2) // TILE + 1
        a, c = min(a, c), max(a, c)
        ia = int(np.searchsorted(b, a, side="right"))
        ic = int(np.searchsorted(b, c, side="right"))
        return int(s2[ia] + a * (s1[ic] - s1[ia]) + a * c * (len(b) - ic))


class ModelBank:
    """Materialized rows of every resident model in one device array [sum K, NP], with the
    host-side pair bounds of their renders.  models: float32 [K_i, NP] materialized rows
    (numpy arrays or tensors).  box: the kernel boxes the renders bin with ("square", the
    boxes the models were fitted with, or "tight"); the pair bound (square boxes) holds for
    both.  mode, trunc: the regression (gated SMoE or the RBF sum of Eq. 1) and the
    truncation reading of the renders (as in make_grid)."""

    def __init__(self, models, C_: int, order: int, radius: float = 3.0, device="cuda",
                 box="square", trunc="gradient", mode="smoe"):
        rows = [m.detach().float().cpu() if torch.is_tensor(m) else
                torch.as_tensor(np.asarray(m, dtype=np.float32)) for m in models]
        for i, r in enumerate(rows):
            if not bool(torch.isfinite(r).all()):
                raise ValueError(f"model {i} holds NaN or infinite parameters")
        self.C, self.order, self.radius = C_, order, float(radius)
        self.box = _box(box)
        self.trunc = _trunc(trunc)
        self.mode = _mode(mode)
        self.K = [int(r.shape[0]) for r in rows]
        self.offset = [int(x) for x in np.concatenate([[0], np.cumsum(self.K)[:-1]])]
        self.params = torch.cat(rows).to(device).contiguous()
        _check_params(self.params, C_, order)
        self.spans = BoxSpans([r.numpy() for r in rows], radius)

    def __len__(self):
        return len(self.K)

    def rows(self, i: int) -> torch.Tensor:
        return self.params[self.offset[i]:self.offset[i] + self.K[i]]

    def pair_bound(self, i: int, scale: int, width: int, height: int,
                   sharpen: float = 1.0) -> int:
        return self.spans.pair_bound(i, scale, width, height, sharpen)


def admit(pending, in_use: int, budget: int, footprint, max_batch: int, max_pixels: int):
    """Admission: pops from the FIFO `pending` the longest head run of requests whose
    footprint(batch) fits `budget - in_use`, at most max_batch requests and (beyond the
    first) max_pixels output pixels.  A request is never skipped for a later one.  Raises
    if the head alone exceeds the whole budget."""
    batch = []
    px = 0
    while pending and len(batch) < max_batch:
        r = pending[0]
        npx = px + r.width * r.height
        if batch and npx > max_pixels:
            break
        need = footprint(batch + [r])
        if in_use + need > budget:
            if not batch and need > budget:
                raise ValueError(f"request needs {need} bytes, over the {budget}-byte budget")
            break
        batch.append(pending.popleft())
        px = npx
    return batch


def _tiles(w: int, h: int, ox: int = 0, oy: int = 0) -> int:
    """Blocks of a raster (16x16 blocks of the output grid aligned to multiples of 16)."""
    return ((ox + w - 1) // TILE - ox // TILE + 1) * ((oy + h - 1) // TILE - oy // TILE + 1)


def _to_requests(reqs):
    return [r if isinstance(r, RenderRequest) else RenderRequest(**r) for r in reqs]


def _summary(results, name: str, extra=None):
    lat = np.array([r.latency for r in results]) * 1e3
    px = sum(r.request.width * r.request.height for r in results)
    t0 = min(r.request.arrival for r in results)
    t1 = max(r.done for r in results)
    wait = np.array([r.started - r.request.arrival for r in results]) * 1e3
    gpu = np.array([r.done - r.started for r in results]) * 1e3
    out = {"server": name, "requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
           "wait_p50_ms": float(np.percentile(wait, 50)), "wait_p99_ms": float(np.percentile(wait, 99)),
           "gpu_p50_ms": float(np.percentile(gpu, 50)), "gpu_p99_ms": float(np.percentile(gpu, 99)),
           "max_ms": float(lat.max()), "pixels": int(px), "makespan_s": float(t1 - t0),
           "pixels_per_s": float(px / max(t1 - t0, 1e-9)),
           "requests_per_s": float(len(results) / max(t1 - t0, 1e-9))}
    if extra:
        out.update(extra)
    return out


class _Clock:
    """Host clock and a reference event: maps device events to host seconds."""

    def __init__(self, stream):
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(stream)
        self.t0 = time.perf_counter()
        self.ref.synchronize()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def at(self, ev) -> float:
        return self.ref.elapsed_time(ev) * 1e-3


class _Hip:
    """The HIP runtime calls the batched loop makes for every batch -- event record, query,
    elapsed time and the status-word copy -- made directly through the runtime torch already
    loaded (each a plain C call, a few microseconds less than torch's wrappers)."""

    _lib = None

    def __init__(self):
        if _Hip._lib is None:
            L = ct.CDLL("libamdhip64.so.7")
            vp = ct.c_void_p
            L.hipEventCreate.argtypes = [ct.POINTER(vp)]
            L.hipEventRecord.argtypes = [vp, vp]
            L.hipEventQuery.argtypes = [vp]
            L.hipEventSynchronize.argtypes = [vp]
            L.hipEventElapsedTime.argtypes = [ct.POINTER(ct.c_float), vp, vp]
            L.hipMemcpyAsync.argtypes = [vp, vp, ct.c_size_t, ct.c_int, vp]
            _Hip._lib = L
        self.L = _Hip._lib

    def event(self) -> int:
        e = ct.c_void_p()
        if self.L.hipEventCreate(ct.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e.value

    def record(self, ev: int, stream: int):
        if self.L.hipEventRecord(ev, stream) != 0:
            raise RuntimeError("hipEventRecord failed")

    def done(self, ev: int) -> bool:
        return self.L.hipEventQuery(ev) == 0  # hipSuccess; hipErrorNotReady while pending

    def sync(self, ev: int):
        if self.L.hipEventSynchronize(ev) != 0:
            raise RuntimeError("hipEventSynchronize failed")

    def elapsed_s(self, a: int, b: int) -> float:
        f = ct.c_float()
        if self.L.hipEventElapsedTime(ct.byref(f), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return f.value * 1e-3

    def copy_d2h(self, dst: int, src: int, n: int, stream: int):
        if self.L.hipMemcpyAsync(dst, src, n, 2, stream) != 0:  # hipMemcpyDeviceToHost
            raise RuntimeError("hipMemcpyAsync failed")


class _HipClock:
    """_Clock with a raw HIP reference event (for the batched loop's raw events)."""

    def __init__(self, hip: _Hip, stream):
        torch.cuda.synchronize()
        self.hip = hip
        self.ref = hip.event()
        hip.record(self.ref, stream.cuda_stream)
        self.t0 = time.perf_counter()
        hip.sync(self.ref)

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def at(self, ev: int) -> float:
        return self.hip.elapsed_s(self.ref, ev)


@contextlib.contextmanager
def _no_gc():
    """The collector paused for a serving run (its pauses would land on request latencies)."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def _wait_until(clock, t):
    while True:
        d = t - clock.now()
        if d <= 0:
            return
        if d > 2e-3:
            time.sleep(d - 1e-3)


@dataclass
class _Batch:
    bid: int
    slot: int
    reqs: list
    nbytes: int
    blocks: int = 0
    start: object = None
    done: object = None
    status_ready: object = None
    status: torch.Tensor | None = None
    keep: list = field(default_factory=list)   # tensors that must live until done
    slices: list = field(default_factory=list)


class _Slot:
    """Per-stream resources reused by every batch the stream runs (a stream runs one batch at
    a time): a pinned staging area and a device copy of the segment table, the batch's
    timing events, and one binning workspace buffer that grows to the largest batch the
    stream has run and is laid out afresh (a host-only call) for each batch."""

    def __init__(self, max_batch: int, device, hip: _Hip):
        self.stream = torch.cuda.Stream()
        self.device = device
        nbytes = max_batch * ct.sizeof(C.SmoeSegment)
        self.table_host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        self.table_dev = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.start, self.done, self.status_ready = hip.event(), hip.event(), hip.event()
        self.ws = torch.empty(0, dtype=torch.uint8, device=device)
        self.bins = C.SmoeBins()
        self.batch = None

    def layout(self, K: int, C_: int, order: int, T: int, P: int) -> C.SmoeBins:
        n = C.smoe_render_workspace_bytes(K, C_, order, T, P)
        if n > self.ws.numel():
            # the old buffer may still be read by this stream's last batch: the caching
            # allocator keeps it until the stream has passed this point
            self.ws.record_stream(self.stream)
            self.ws = torch.empty(max(n, 2 * self.ws.numel()), dtype=torch.uint8,
                                  device=self.device)
        C.smoe_render_workspace_layout(self.bins, self.ws.data_ptr(), self.ws.numel(), K, C_,
                                       order, T, P)
        return self.bins


def _check(hip, bt):
    hip.sync(bt.status_ready)
    if int(bt.status[1]) != 0:
        raise RuntimeError("pair bound exceeded: a batch overflowed its workspace")


class Server:
    """Continuous batching over `streams` streams under an HBM budget (bytes)."""

    def __init__(self, bank: ModelBank, budget_bytes: int = 8 << 30, streams: int = 2,
                 max_batch: int = 32, max_batch_pixels: int = 1 << 26,
                 fill_blocks: int = 4096, overlap_backlog: int = 2, reserve_for=None):
        """fill_blocks: a further batch is started beside those in flight only while they
        hold fewer 16x16 blocks than this -- about half of what the GPU renders at once
        (256 CUs x 4 SIMDs x 7-8 one-wave blocks).  A batch that fills the GPU runs alone;
        requests that arrive meanwhile queue and leave together in the next batch.
        overlap_backlog: a batch is started beside one in flight only when at least this many
        requests wait; a lone request waits for the batch in flight instead (measured: at
        light load, overlapping a lone request lengthens the tail of the larger renders).
        reserve_for: optional (width, height, scales) of the largest requests to expect: every
        stream's workspace is then sized up front for the largest of them on any resident
        model, so that no request pays for growing it."""
        if streams < 1 or max_batch < 1:
            raise ValueError("at least one stream and one request per batch")
        self.fill_blocks = int(fill_blocks)
        self.overlap_backlog = max(1, int(overlap_backlog))
        self.bank = bank
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_batch_pixels = int(max_batch_pixels)
        self.nbytes_px = 4 * bank.C
        self.hip = _Hip()
        self.slots = [_Slot(self.max_batch, bank.params.device, self.hip) for _ in range(streams)]
        # pinned status words of recent batches (a ring: a row is read before it is reused)
        self._status = torch.zeros((256, 4), dtype=torch.int32, pin_memory=True)
        self.streams = [sl.stream for sl in self.slots]
        self._models = [model_struct(bank.rows(i), bank.C, bank.order) for i in range(len(bank))]
        # per request shape (model, size, scale, window origin, sharpening): its kernels,
        # blocks, pair bound, pixels and bytes -- a request's shape recurs, its bound need
        # not be recomputed on the path to its launch
        self._shape_info = {}
        if reserve_for is not None:
            w, h, scales = reserve_for
            t = _tiles(w, h, TILE - 1, TILE - 1)  # the most blocks such a window touches
            shapes = [(bank.K[i], t, bank.pair_bound(i, s, w, h)) for i in range(len(bank))
                      for s in scales]
            for sl in self.slots:
                for k, tt, p in shapes:
                    sl.layout(k, bank.C, bank.order, tt, p)

    def _info(self, r):
        """(kernels, blocks, pair bound, pixels, bytes alone) of one request, computed once per
        request shape."""
        inf = getattr(r, "_smoe_info", None)
        if inf is None:
            key = (r.model, r.scale, r.width, r.height, r.origin_x, r.origin_y, r.sharpen)
            inf = self._shape_info.get(key)
            if inf is None:
                k, t = self.bank.K[r.model], _tiles(r.width, r.height, r.origin_x, r.origin_y)
                p = self.bank.pair_bound(r.model, r.scale, r.width, r.height, r.sharpen)
                n = r.width * r.height
                nbytes = (C.smoe_render_workspace_bytes(k, self.bank.C, self.bank.order, t, p)
                          + n * self.nbytes_px + 64)
                inf = (k, t, p, n, nbytes)
                if len(self._shape_info) >= 4096:
                    self._shape_info.clear()
                self._shape_info[key] = inf
            r._smoe_info = inf
        return inf

    def footprint(self, reqs) -> tuple[int, int, int, int]:
        """(bytes, kernels, blocks, pair bound) of one batch of requests."""
        K = T = P = px = 0
        for r in reqs:
            k, t, p, n, _ = self._info(r)
            K, T, P, px = K + k, T + t, P + p, px + n
        ws = C.smoe_render_workspace_bytes(K, self.bank.C, self.bank.order, T, P)
        return ws + px * self.nbytes_px + 64 * len(reqs), K, T, P

    def _launch(self, batch: _Batch, keep_outputs: bool, K: int, T: int, P: int):
        b = self.bank
        sl = self.slots[batch.slot]
        st = sl.stream
        dev = b.params.device
        hip = self.hip
        with torch.cuda.stream(st):
            batch.start = sl.start
            hip.record(batch.start, st.cuda_stream)
            bins = sl.layout(K, b.C, b.order, T, P)
            if len(batch.reqs) == 1:
                # one request: the single-raster calls, no segment table
                r = batch.reqs[0]
                grid = make_grid(r.width, r.height, r.scale, r.origin_x, r.origin_y, b.radius,
                                 r.sharpen, b.box, mode=b.mode, trunc=b.trunc)
                m = self._models[r.model]
                # the binning goes first, so that the device starts while the host allocates
                # the output
                C.smoe_bin(m, grid, bins, st.cuda_stream)
                images = torch.empty((r.height * r.width, b.C), dtype=torch.float32, device=dev)
                C.smoe_render(m, grid, bins, images.data_ptr(), None, None, None, st.cuda_stream)
                slices = [(0, r.height * r.width, r.height, r.width)]
            else:
                n = len(batch.reqs)
                host = (C.SmoeSegment * n).from_address(sl.table_host.data_ptr())
                for sg, r in zip(host, batch.reqs):
                    sg.width, sg.height, sg.scale = r.width, r.height, r.scale
                    sg.origin_x, sg.origin_y = r.origin_x, r.origin_y
                    sg.sharpen = r.sharpen
                    sg.num_kernels, sg.param_offset = b.K[r.model], b.offset[r.model]
                _, _, npx = C.smoe_segments_layout(host)
                nb = n * ct.sizeof(C.SmoeSegment)
                sl.table_dev[:nb].copy_(sl.table_host[:nb], non_blocking=True)
                images = torch.empty((npx, b.C), dtype=torch.float32, device=dev)
                cb = C.SmoeBatch(b.C, b.order, b.params.data_ptr(), b.params.shape[0], n,
                                 sl.table_dev.data_ptr(), ct.addressof(host), b.radius, b.box,
                                 b.mode, b.trunc)
                C.smoe_bin_batched(cb, bins, st.cuda_stream)
                C.smoe_render_batched(cb, bins, images.data_ptr(), None, st.cuda_stream)
                slices = [(sg.pixel_offset, sg.pixel_offset + sg.width * sg.height, sg.height,
                           sg.width) for sg in host]
            # the images are complete at `done`; the status words follow and are checked once
            # their copy has landed (the batch's slot is released at `done`)
            batch.done = sl.done
            hip.record(batch.done, st.cuda_stream)
            batch.status = self._status[batch.bid % len(self._status)]
            hip.copy_d2h(batch.status.data_ptr(), bins.status, 16, st.cuda_stream)
            batch.status_ready = sl.status_ready
            hip.record(batch.status_ready, st.cuda_stream)
        batch.keep = [images]
        if keep_outputs:
            batch.slices = [images[a:e].view(h, w, b.C) for a, e, h, w in slices]

    def serve(self, requests, realtime: bool = True, keep_outputs: bool = False):
        """Serves every request; returns (results in request order, summary dict).  With
        realtime=False every request is taken as arrived at time 0 (saturation)."""
        with _no_gc():
            return self._serve(requests, realtime, keep_outputs)

    def _serve(self, requests, realtime, keep_outputs):
        reqs = _to_requests(requests)
        if not realtime:
            reqs = [RenderRequest(**{**r.__dict__, "arrival": 0.0}) for r in reqs]
        order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
        results = [None] * len(reqs)
        index = {id(r): i for i, r in enumerate(reqs)}
        pending = deque()
        free = list(range(len(self.slots)))
        inflight = 0
        inflight_blocks = 0
        in_use = peak = 0
        nxt = nb = 0
        sizes = []
        checks = []  # finished batches whose status words are still to be read
        hip = self.hip
        clock = _HipClock(hip, self.streams[0])
        footprint = lambda q: self.footprint(q)[0]  # noqa: E731
        while nxt < len(order) or pending or inflight:
            now = clock.now()
            while nxt < len(order) and reqs[order[nxt]].arrival <= now:
                r = reqs[order[nxt]]
                self._info(r)
                pending.append(r)
                nxt += 1
            if inflight:
                for si, sl in enumerate(self.slots):
                    bt = sl.batch
                    if bt is None or not hip.done(bt.done):
                        continue
                    t = clock.at(bt.done)
                    t_start = clock.at(bt.start)
                    bt.keep = []  # later work on this stream may reuse the memory
                    checks.append(bt)
                    for j, r in enumerate(bt.reqs):
                        results[index[id(r)]] = RenderResult(
                            r, t, bt.bid, bt.slices[j] if keep_outputs else None, t_start)
                    in_use -= bt.nbytes
                    inflight_blocks -= bt.blocks
                    sl.batch = None
                    free.append(si)
                    inflight -= 1
            while (free and pending and inflight_blocks < self.fill_blocks
                   and (not inflight or len(pending) >= self.overlap_backlog)):
                if len(pending) == 1:  # the common case at low load
                    k, t, p, _, need = pending[0]._smoe_info
                    if in_use + need > self.budget:
                        if need > self.budget:
                            raise ValueError(f"request needs {need} bytes, over the budget")
                        break
                    got = [pending.popleft()]
                    shape = (k, t, p)
                else:
                    got = admit(pending, in_use, self.budget, footprint, self.max_batch,
                                self.max_batch_pixels)
                    if not got:
                        break
                    need, k, t, p = self.footprint(got)
                    shape = (k, t, p)
                while checks and checks[0].bid <= nb - len(self._status):
                    _check(hip, checks.pop(0))  # its status row is about to be reused
                si = min(free)  # the lowest free stream: at low load always the same one
                free.remove(si)
                bt = _Batch(nb, si, got, need, blocks=shape[1])
                nb += 1
                self._launch(bt, keep_outputs, *shape)
                self.slots[si].batch = bt
                inflight += 1
                inflight_blocks += bt.blocks
                in_use += need
                peak = max(peak, in_use)
                sizes.append(len(got))
            if not inflight and not pending and nxt < len(order):
                _wait_until(clock, reqs[order[nxt]].arrival)
        torch.cuda.synchronize()
        for bt in checks:
            _check(hip, bt)
        return results, _summary(results, "batched", {
            "batches": nb, "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "max_batch": int(max(sizes)) if sizes else 0, "streams": len(self.slots),
            "fill_blocks": self.fill_blocks, "overlap_backlog": self.overlap_backlog,
            "peak_bytes": int(peak), "budget_bytes": self.budget})


class PlainServer:
    """One launch sequence (bin, render) per request on one stream, host-synchronised."""

    def __init__(self, bank: ModelBank):
        self.bank = bank
        self.stream = torch.cuda.Stream()

    def serve(self, requests, realtime: bool = True, keep_outputs: bool = False):
        with _no_gc():
            return self._serve(requests, realtime, keep_outputs)

    def _serve(self, requests, realtime, keep_outputs):
        b = self.bank
        reqs = _to_requests(requests)
        if not realtime:
            reqs = [RenderRequest(**{**r.__dict__, "arrival": 0.0}) for r in reqs]
        order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
        results = [None] * len(reqs)
        st = self.stream
        clock = _Clock(st)
        for i in order:
            r = reqs[i]
            _wait_until(clock, r.arrival)
            grid = make_grid(r.width, r.height, r.scale, r.origin_x, r.origin_y, b.radius,
                             r.sharpen, b.box, mode=b.mode, trunc=b.trunc)
            rows = b.rows(r.model)
            m = model_struct(rows, b.C, b.order)
            with torch.cuda.stream(st):
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(st)
                bins = Bins(b.K[r.model], b.C, b.order,
                            _tiles(r.width, r.height, r.origin_x, r.origin_y),
                            b.pair_bound(r.model, r.scale, r.width, r.height, r.sharpen),
                            device=rows.device, render_only=True, zero=False)
                image = torch.empty((r.height, r.width, b.C), dtype=torch.float32,
                                    device=rows.device)
                C.smoe_bin(m, grid, bins.c, st.cuda_stream)
                C.smoe_render(m, grid, bins.c, image.data_ptr(), None, None, None, st.cuda_stream)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(st)
            code, status = C.smoe_read_status(bins.c, st.cuda_stream)
            if code == C.SMOE_ERR_CAPACITY:
                raise RuntimeError("pair bound exceeded: request overflowed its workspace")
            results[i] = RenderResult(r, clock.at(ev), i, image if keep_outputs else None,
                                      clock.at(ev0))
        torch.cuda.synchronize()
        return results, _summary(results, "plain")


def latency_table(summaries) -> str:
    """A small text table of serving summaries."""
    keys = ["server", "requests", "p50_ms", "p99_ms", "mean_ms", "pixels_per_s"]
    lines = [" | ".join(keys)]
    for s in summaries:
        lines.append(" | ".join(f"{s[k]:.4g}" if isinstance(s[k], float) else str(s[k])
                                for k in keys))
    return "\n".join(lines)


__all__ = ["RenderRequest", "RenderResult", "BoxSpans", "ModelBank", "admit", "Server",
           "PlainServer", "latency_table"]
