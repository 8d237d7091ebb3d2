"""ctypes front end of the plain FP64 CPU oracle (``smoe_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may use this module; the product path (the HIP library and its
Python binding) never imports it.

All model arrays are float64 rows in the layouts documented in
``smoe_oracle.cpp`` (materialized: mu_x, mu_y, l11, l21, l22, rho, a, wx, wy;
raw: mu_x, mu_y, s1, l21, s2, rho, a, wx, wy).  float32 inputs are widened
exactly.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from pathlib import Path

import numpy as np

_DIR = Path(__file__).resolve().parent
_SRC = _DIR / "smoe_oracle.cpp"
_LIB = _DIR / "liboracle.so"

# -ffp-contract=off: the binary32 truncation rule must be evaluated op by op, with
# no fused multiply-adds.  No -march: the library must run on any x86-64 host.
CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
            "-pthread"]


def build(force: bool = True) -> Path:
    """Compile the oracle into ``oracle/liboracle.so``."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call(["g++", *CXXFLAGS, str(_SRC), "-o", str(tmp)])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_path = None


def use_library(path=None):
    """Bind to another build of the oracle source (tests that plant mistakes in a copy);
    None restores the default library."""
    global _lib, _lib_path
    _lib, _lib_path = None, (None if path is None else Path(path))


def lib():
    global _lib
    if _lib is None:
        path = _lib_path or _LIB
        if path == _LIB and not _LIB.exists():
            build()
        L = ct.CDLL(str(path))
        dp, fp = ct.POINTER(ct.c_double), ct.POINTER(ct.c_float)
        i32p, u32p = ct.POINTER(ct.c_int32), ct.POINTER(ct.c_uint32)
        I, F, D, I64 = ct.c_int, ct.c_float, ct.c_double, ct.c_int64
        L.oracle_num_params.argtypes = [I, I]
        L.oracle_num_params.restype = I
        L.oracle_bin.argtypes = [I, I, I, dp, I, I, I, I, I, F, I, I, i32p, i32p, i32p, I64, u32p, u32p, i32p]
        L.oracle_bin.restype = I64
        L.oracle_render.argtypes = [I, I, I, dp, I, I, I, I, I, F, I, I, I, I, I64, i32p, dp, dp, I]
        L.oracle_render.restype = None
        L.oracle_render_points.argtypes = [I, I, I, dp, F, I, I, I, I, I64, fp, dp, dp, I]
        L.oracle_render_points.restype = None
        L.oracle_loss_grad.argtypes = [I, I, I, dp, I, I, I, I, I, F, I, I, I, dp, dp, I, i32p, dp, I]
        L.oracle_loss_grad.restype = D
        L.oracle_materialize.argtypes = [I, I, I, dp, dp]
        L.oracle_materialize.restype = None
        L.oracle_step_lrs.argtypes = [I, I, D, D, D, D, D, dp]
        L.oracle_step_lrs.restype = None
        L.oracle_adam.argtypes = [I, I, I, dp, dp, dp, dp, I, dp, D, D, D]
        L.oracle_adam.restype = None
        L.oracle_fit.argtypes = [I, I, I, dp, I, I, F, I, I, I, dp, I, I, D, D, D, D, D, D, D, D, dp, dp, I]
        L.oracle_fit.restype = None
        _lib = L
    return _lib


def default_threads() -> int:
    n = os.environ.get("OMP_NUM_THREADS")
    if n and n.isdigit() and int(n) > 0:
        return min(int(n), os.cpu_count() or 1)
    return os.cpu_count() or 1


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(ct.POINTER(t))


def _trunc(trunc) -> int:
    return {"render": 0, "gradient": 1}[trunc]


def num_params(C: int, order: int) -> int:
    return int(lib().oracle_num_params(C, order))


def _KC(model, C, order):
    model = _d(model)
    NP = num_params(C, order)
    assert model.ndim == 2 and model.shape[1] == NP, (model.shape, NP)
    return model, model.shape[0]


def bin(model, C, order, W, H, s=1, ox=0, oy=0, r=3.0, capacity=None, box=0, trunc="gradient"):
    """Block lists.  Returns dict(tile_rects, native_rects, counts, P, keys, vals, ranges):
    tile_rects are output blocks of the raster, native_rects the kernels' native 16x16 blocks
    clamped to those the raster's sample points reach.
    box: 0 = the square box of Sec. IV-B, 1 = the tight axis-aligned box.  trunc: the reading
    ("gradient": native blocks holding a pixel centre in the box; "render": blocks the box
    overlaps)."""
    model, K = _KC(model, C, order)
    T = blocks(W, ox) * blocks(H, oy)
    tr = np.zeros((K, 4), np.int32)
    pr = np.zeros((K, 4), np.int32)
    cnt = np.zeros(K, np.int32)
    rng = np.zeros((T, 2), np.int32)
    if capacity is None:
        P = lib().oracle_bin(K, C, order, _ptr(model, ct.c_double), W, H, s, ox, oy, r, box,
                             _trunc(trunc), _ptr(tr, ct.c_int32), _ptr(pr, ct.c_int32), _ptr(cnt, ct.c_int32),
                             0, None, None, _ptr(rng, ct.c_int32))
        capacity = P
    keys = np.zeros(max(capacity, 1), np.uint32)
    vals = np.zeros(max(capacity, 1), np.uint32)
    P = lib().oracle_bin(K, C, order, _ptr(model, ct.c_double), W, H, s, ox, oy, r, box,
                         _trunc(trunc), _ptr(tr, ct.c_int32), _ptr(pr, ct.c_int32), _ptr(cnt, ct.c_int32),
                         capacity, _ptr(keys, ct.c_uint32), _ptr(vals, ct.c_uint32),
                         _ptr(rng, ct.c_int32))
    n = min(P, capacity)
    return dict(tile_rects=tr, native_rects=pr, counts=cnt, P=int(P), keys=keys[:n],
                vals=vals[:n], ranges=rng)


def blocks(n: int, o: int = 0) -> int:
    """Blocks along an axis of n output pixels at origin o: the 16-pixel blocks of the output
    grid, aligned to multiples of 16 in o + u, that the pixels touch."""
    return (o + n - 1) // 16 - o // 16 + 1


def _truncated(truncated) -> int:
    """True / 1: the truncation rule; False / 0: every kernel (the global model of Sec.
    III-B); "lists" / 2: every kernel of the point's block list, with no cut."""
    if truncated == "lists":
        return 2
    t = int(truncated)
    assert t in (0, 1, 2), truncated
    return t


def render(model, C, order, W, H, s=1, ox=0, oy=0, r=3.0, truncated=True, pixels=None,
           threads=None, box=0, rbf=False, trunc="gradient"):
    """y [H, W, C] and D [H, W] (or [n, C], [n] at the listed (u, v) pixels).  rbf: the
    weighted sum of kernels of Eq. (1) instead of the gated regression of Eq. (2)-(4).
    trunc: "gradient" (the render takes every representable term of the block's list; the
    ellipse test applies to gradients only -- Sec. IV-B) or "render" (the ellipse test
    applies to the render as well).  truncated: see _truncated."""
    model, K = _KC(model, C, order)
    threads = threads or default_threads()
    if pixels is None:
        y = np.zeros((H, W, C), np.float64)
        D = np.zeros((H, W), np.float64)
        lib().oracle_render(K, C, order, _ptr(model, ct.c_double), W, H, s, ox, oy, r, box, int(rbf),
                            _trunc(trunc), _truncated(truncated), 0, None, _ptr(y, ct.c_double), _ptr(D, ct.c_double),
                            threads)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
        y = np.zeros((pix.shape[0], C), np.float64)
        D = np.zeros(pix.shape[0], np.float64)
        lib().oracle_render(K, C, order, _ptr(model, ct.c_double), W, H, s, ox, oy, r, box, int(rbf),
                            _trunc(trunc), _truncated(truncated), pix.shape[0], _ptr(pix, ct.c_int32),
                            _ptr(y, ct.c_double), _ptr(D, ct.c_double), threads)
    return y, D


def render_points(model, C, order, points, r=3.0, truncated=True, threads=None, box=0,
                  rbf=False, trunc="gradient"):
    """y [n, C] and D [n] at arbitrary native points (float32 [n, 2] = (x, y)), with the
    kernels' boxes on the native block grid: the regression itself, independent of any
    raster."""
    model, K = _KC(model, C, order)
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 2)
    n = pts.shape[0]
    y = np.zeros((n, C), np.float64)
    D = np.zeros(n, np.float64)
    lib().oracle_render_points(K, C, order, _ptr(model, ct.c_double), r, box, int(rbf),
                               _trunc(trunc), _truncated(truncated), n, _ptr(pts, ct.c_float),
                               _ptr(y, ct.c_double), _ptr(D, ct.c_double),
                               threads or default_threads())
    return y, D


def sample_points(W, H, s=1, ox=0, oy=0):
    """float32 [H, W, 2] native sample points of an output raster: ((o + u) + 0.5) * (1/s),
    with 1/s rounded to binary32 once."""
    inv = np.float32(1.0) / np.float32(s)
    xs = ((np.arange(W) + ox).astype(np.float32) + np.float32(0.5)) * inv
    ys = ((np.arange(H) + oy).astype(np.float32) + np.float32(0.5)) * inv
    P = np.zeros((H, W, 2), np.float32)
    P[..., 0] = xs[None, :]
    P[..., 1] = ys[:, None]
    return P


def loss_grad(model, C, order, W, H, target=None, grad_y=None, kernels=None, s=1, ox=0, oy=0,
              r=3.0, threads=None, box=0, rbf=False, trunc="gradient"):
    """(loss, grads [K or len(kernels), NP]) in raw-parameter order."""
    model, K = _KC(model, C, order)
    NP = model.shape[1]
    assert (target is None) != (grad_y is None)
    t = None if target is None else _d(target).reshape(H, W, C)
    gy = None if grad_y is None else _d(grad_y).reshape(H, W, C)
    sel = None if kernels is None else np.ascontiguousarray(kernels, dtype=np.int32)
    nout = K if sel is None else sel.shape[0]
    g = np.zeros((nout, NP), np.float64)
    loss = lib().oracle_loss_grad(K, C, order, _ptr(model, ct.c_double), W, H, s, ox, oy, r, box, int(rbf),
                                  _trunc(trunc), _ptr(t, ct.c_double), _ptr(gy, ct.c_double),
                                  0 if sel is None else sel.shape[0], _ptr(sel, ct.c_int32),
                                  _ptr(g, ct.c_double), threads or default_threads())
    return float(loss), g


def sharpen(model, f):
    """Native sharpening by kernel editing (Sec. II-B; the sharpened super-resolution of
    Sec. V-D): every kernel's bandwidth is reduced by the factor f, i.e. the Cholesky factor
    L of its covariance becomes L / f (Sigma -> Sigma / f^2); centres, gating weights and
    experts are unchanged.  The division is taken in binary32 (the precision the model rows
    and the truncation rule are decided in), so the edited rows are exactly the rows a
    binary32 renderer sees.  f = 1 (or 0) returns the model unchanged."""
    model = _d(model).copy()
    f = float(f)
    if f not in (0.0, 1.0):
        L = model[:, 2:5].astype(np.float32)
        model[:, 2:5] = (L / np.float32(f)).astype(np.float64)
    return model


def materialize(raw, C, order):
    raw, K = _KC(raw, C, order)
    out = np.zeros_like(raw)
    lib().oracle_materialize(K, C, order, _ptr(raw, ct.c_double), _ptr(out, ct.c_double))
    return out


def step_lrs(step_index, total_steps, lr_mu, lr_mu_final, lr_chol, lr_rho, lr_expert):
    out = np.zeros(4, np.float64)
    lib().oracle_step_lrs(step_index, total_steps, lr_mu, lr_mu_final, lr_chol, lr_rho,
                          lr_expert, _ptr(out, ct.c_double))
    return out


def adam(p, g, m, v, t, lrs4, C, order, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays p, m, v (gradient g), 1-based step t."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _d(g)
    lrs4 = _d(lrs4)
    K = p.shape[0]
    lib().oracle_adam(K, C, order, _ptr(p, ct.c_double), _ptr(g, ct.c_double),
                      _ptr(m, ct.c_double), _ptr(v, ct.c_double), t, _ptr(lrs4, ct.c_double),
                      beta1, beta2, eps)


def fit(raw0, C, order, target, steps, total_steps=None, lr_mu=1e-2, lr_mu_final=None,
        lr_chol=1e-2, lr_rho=1e-2, lr_expert=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, r=3.0,
        threads=None, box=0, rbf=False, trunc="gradient"):
    """FP64 fit.  Returns (loss history [steps], final raw params [K, NP])."""
    raw0, K = _KC(raw0, C, order)
    t = _d(target)
    H, W = t.shape[:2]
    hist = np.zeros(steps, np.float64)
    out = np.zeros_like(raw0)
    lib().oracle_fit(K, C, order, _ptr(raw0, ct.c_double), W, H, r, box, int(rbf), _trunc(trunc),
                     _ptr(t, ct.c_double),
                     steps,
                     total_steps or steps, lr_mu, lr_mu if lr_mu_final is None else lr_mu_final,
                     lr_chol, lr_rho, lr_expert, beta1, beta2, eps, _ptr(hist, ct.c_double),
                     _ptr(out, ct.c_double), threads or default_threads())
    return hist, out


def window_rects(H, W, d, window=16):
    """The windows of the multi-model estimator (Sec. V-C): window-sized squares shifted by d
    over the image, placed so that every pixel has the same number of windows covering it --
    window / d along each axis; the first window therefore starts window - d pixels before the
    image -- and clipped to the image.  [(y0, x0, h, w)], window rows top to bottom, each row
    left to right.  Each axis is enumerated by brute force: every start that reaches into
    the image."""
    assert window % d == 0

    def spans(n):
        out = []
        for start in range(-(window - d), n, d):
            cover = [p for p in range(start, start + window) if 0 <= p < n]
            out.append((cover[0], len(cover)))
        return out

    return [(y0, x0, h, w) for (y0, h) in spans(H) for (x0, w) in spans(W)]


def fuse_windows(models, C, order, H, W, d, window=16, r=3.0, trunc="gradient", threads=None):
    """The multi-model estimate of Eq. (10)-(11): at each pixel, the mean of the predictions
    y_h of the window models h whose window covers it.  models: one model (rows) per window
    of window_rects(H, W, d, window), in that order, each in its window's own pixel
    coordinates (the window's top-left pixel at (0, 0)).  Each window model is rendered on
    its window's raster by render(); the sum and the count run in float64.  Returns y
    [H, W, C] float64."""
    rects = window_rects(H, W, d, window)
    assert len(models) == len(rects), "one model per window"
    acc = np.zeros((H, W, C), np.float64)
    cnt = np.zeros((H, W), np.float64)
    for (y0, x0, h, w), model in zip(rects, models):
        y, _ = render(model, C, order, w, h, r=r, trunc=trunc, threads=threads)
        acc[y0:y0 + h, x0:x0 + w] += y
        cnt[y0:y0 + h, x0:x0 + w] += 1.0
    return acc / cnt[..., None]
