"""ctypes binding of the C ABI in ``include/smoe.h`` (``libsmoe.so``).

Argument marshalling only: every step of the SMoE path runs in the library's HIP
kernels.  The structures below mirror the C structs field for field; functions
keep the C names.  There is no CPU fallback: importing this module without the
built library raises ImportError.
"""
from __future__ import annotations

import ctypes as ct
from pathlib import Path

# torch first: it loads its HIP runtime (libamdhip64.so.7), and libsmoe.so, whose dependency
# carries the same soname, then binds to that one.  Loaded the other way round the process
# would hold two HIP runtimes, and the library's could see a different set of devices than
# the one that owns torch's memory and streams.
import torch  # noqa: F401,E402

_LIB_PATH = Path(__file__).resolve().parent / "libsmoe.so"

SMOE_OK = 0
SMOE_ERR_INVALID = -1
SMOE_ERR_CAPACITY = -2
SMOE_ERR_HIP = -3
SMOE_ERR_TOO_LARGE = -4
SMOE_ERR_NONFINITE = -5

SMOE_BOX_SQUARE = 0
SMOE_BOX_TIGHT = 1
SMOE_MODE_SMOE = 0
SMOE_MODE_RBF = 1
SMOE_TRUNC_GRADIENT = 0
SMOE_TRUNC_RENDER = 1
TILE = 16

_i32, _f32, _vp, _sz = ct.c_int32, ct.c_float, ct.c_void_p, ct.c_size_t


class SmoeModel(ct.Structure):
    _fields_ = [("K", _i32), ("C", _i32), ("order", _i32), ("params", _vp)]


class SmoeGrid(ct.Structure):
    _fields_ = [("width", _i32), ("height", _i32), ("scale", _i32), ("origin_x", _i32),
                ("origin_y", _i32), ("radius", _f32), ("sharpen", _f32),
                ("box", _i32), ("mode", _i32), ("trunc", _i32)]


class SmoeSegment(ct.Structure):
    _fields_ = [("width", _i32), ("height", _i32), ("scale", _i32), ("origin_x", _i32),
                ("origin_y", _i32), ("num_kernels", _i32), ("param_offset", _i32),
                ("kernel_offset", _i32), ("tile_offset", _i32), ("sharpen", _f32),
                ("pixel_offset", ct.c_int64)]


class SmoeBatch(ct.Structure):
    _fields_ = [("C", _i32), ("order", _i32), ("params", _vp), ("num_params_rows", _i32),
                ("num_segments", _i32), ("segments", _vp), ("segments_host", _vp),
                ("radius", _f32), ("box", _i32), ("mode", _i32), ("trunc", _i32)]


class SmoeBins(ct.Structure):
    _fields_ = [("K", _i32), ("C", _i32), ("order", _i32), ("max_tiles", _i32),
                ("capacity", _i32), ("tile_rects", _vp), ("native_rects", _vp), ("counts", _vp), ("records", _vp),
                ("record_stride", _i32), ("tile_counts", _vp), ("ranges", _vp), ("keys", _vp),
                ("vals", _vp), ("vals_alt", _vp), ("pair_grads", _vp),
                ("tile_loss", _vp),
                ("status", _vp)]


class SmoeAdamConfig(ct.Structure):
    _fields_ = [("lr_mu", _f32), ("lr_mu_final", _f32), ("lr_chol", _f32), ("lr_rho", _f32),
                ("lr_expert", _f32), ("beta1", _f32), ("beta2", _f32), ("eps", _f32),
                ("total_steps", _i32)]


class SmoeFitState(ct.Structure):
    _fields_ = [("K", _i32), ("C", _i32), ("order", _i32), ("grid", SmoeGrid),
                ("adam", SmoeAdamConfig), ("raw", _vp), ("adam_m", _vp), ("adam_v", _vp),
                ("model", _vp), ("grads", _vp), ("image", _vp), ("denom", _vp),
                ("loss_history", _vp), ("max_steps", _i32), ("prepared", _i32),
                ("write_render", _i32), ("step", _vp),
                ("scalars", _vp), ("num_segments", _i32), ("segments", _vp),
                ("segments_host", _vp), ("bins", SmoeBins)]


class SmoeError(RuntimeError):
    def __init__(self, fn: str, code: int):
        names = {SMOE_ERR_INVALID: "SMOE_ERR_INVALID", SMOE_ERR_CAPACITY: "SMOE_ERR_CAPACITY",
                 SMOE_ERR_HIP: "SMOE_ERR_HIP", SMOE_ERR_TOO_LARGE: "SMOE_ERR_TOO_LARGE",
                 SMOE_ERR_NONFINITE: "SMOE_ERR_NONFINITE"}
        msg = f"{fn} failed: {names.get(code, code)}"
        if code == SMOE_ERR_HIP:
            try:
                msg += f" ({lib.smoe_last_error().decode()})"
            except Exception:  # noqa: BLE001  (the message is best effort)
                pass
        super().__init__(msg)
        self.code = code


def _load():
    if not _LIB_PATH.exists():
        raise ImportError(
            f"{_LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "(the SMoE path has no CPU fallback)")
    L = ct.CDLL(str(_LIB_PATH))
    P = ct.POINTER
    L.smoe_version.argtypes = []
    L.smoe_version.restype = _i32
    L.smoe_bins_workspace_bytes.argtypes = [_i32, _i32, _i32, _i32, _i32]
    L.smoe_bins_workspace_bytes.restype = _sz
    L.smoe_bins_layout.argtypes = [P(SmoeBins), _vp, _sz, _i32, _i32, _i32, _i32, _i32]
    L.smoe_bins_layout.restype = _i32
    L.smoe_render_workspace_bytes.argtypes = [_i32, _i32, _i32, _i32, _i32]
    L.smoe_render_workspace_bytes.restype = _sz
    L.smoe_render_workspace_layout.argtypes = [P(SmoeBins), _vp, _sz, _i32, _i32, _i32, _i32, _i32]
    L.smoe_render_workspace_layout.restype = _i32
    L.smoe_bin.argtypes = [P(SmoeModel), P(SmoeGrid), P(SmoeBins), _vp]
    L.smoe_bin.restype = _i32
    L.smoe_render.argtypes = [P(SmoeModel), P(SmoeGrid), P(SmoeBins), _vp, _vp, _vp, _vp, _vp]
    L.smoe_render.restype = _i32
    L.smoe_render_backward.argtypes = [P(SmoeModel), P(SmoeGrid), P(SmoeBins), _vp, _vp, _vp,
                                       _vp, _vp, _vp]
    L.smoe_render_backward.restype = _i32
    L.smoe_materialize.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp]
    L.smoe_materialize.restype = _i32
    L.smoe_fit_step.argtypes = [P(SmoeFitState), _vp, _vp, _vp]
    L.smoe_fit_step.restype = _i32
    L.smoe_fit_step_timed.argtypes = [P(SmoeFitState), _vp, _vp, P(_vp), _vp]
    L.smoe_fit_step_timed.restype = _i32
    L.smoe_pair_stats.argtypes = [P(SmoeModel), P(SmoeGrid), P(SmoeBins), _vp, _vp]
    L.smoe_pair_stats.restype = _i32
    L.smoe_last_error.argtypes = []
    L.smoe_last_error.restype = ct.c_char_p
    L.smoe_read_status.argtypes = [P(SmoeBins), P(_i32), _vp]
    L.smoe_read_status.restype = _i32
    L.smoe_segments_layout.argtypes = [P(SmoeSegment), _i32, P(_i32), P(_i32), P(ct.c_int64)]
    L.smoe_segments_layout.restype = _i32
    L.smoe_bin_batched.argtypes = [P(SmoeBatch), P(SmoeBins), _vp]
    L.smoe_bin_batched.restype = _i32
    L.smoe_render_batched.argtypes = [P(SmoeBatch), P(SmoeBins), _vp, _vp, _vp]
    L.smoe_render_batched.restype = _i32
    L.smoe_fit_segment_losses.argtypes = [P(SmoeFitState), _vp, _vp]
    L.smoe_fit_segment_losses.restype = _i32
    L.smoe_render_noalloc.argtypes = [P(SmoeModel), P(SmoeGrid), _vp, _vp, _vp, _vp]
    L.smoe_render_noalloc.restype = _i32
    L.smoe_fuse_windows.argtypes = [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp]
    L.smoe_fuse_windows.restype = _i32
    L.smoe_issue_probe.argtypes = [_i32, _i32, _i32, _vp, _vp]
    L.smoe_issue_probe.restype = _i32
    return L


lib = _load()

# Symbols the header declares; the CPU test suite checks that each is exported.
EXPORTED = ["smoe_version", "smoe_bins_workspace_bytes", "smoe_bins_layout", "smoe_bin",
            "smoe_render", "smoe_render_backward", "smoe_materialize", "smoe_fit_step",
            "smoe_fit_step_timed", "smoe_pair_stats", "smoe_read_status", "smoe_segments_layout",
            "smoe_bin_batched", "smoe_render_batched", "smoe_fit_segment_losses",
            "smoe_render_workspace_bytes", "smoe_render_workspace_layout", "smoe_last_error",
            "smoe_render_noalloc", "smoe_fuse_windows", "smoe_issue_probe"]


def _check(fn: str, code: int, allow=()):
    if code != SMOE_OK and code not in allow:
        raise SmoeError(fn, code)
    return code


def smoe_version() -> int:
    return int(lib.smoe_version())


def smoe_bins_workspace_bytes(K, C, order, max_tiles, capacity) -> int:
    return int(lib.smoe_bins_workspace_bytes(K, C, order, max_tiles, capacity))


def smoe_bins_layout(bins: SmoeBins, workspace_ptr: int, nbytes: int, K, C, order, max_tiles,
                     capacity):
    return _check("smoe_bins_layout",
                  lib.smoe_bins_layout(ct.byref(bins), workspace_ptr, nbytes, K, C, order,
                                       max_tiles, capacity))


def smoe_render_workspace_bytes(K, C, order, max_tiles, capacity) -> int:
    return int(lib.smoe_render_workspace_bytes(K, C, order, max_tiles, capacity))


def smoe_render_workspace_layout(bins: SmoeBins, workspace_ptr: int, nbytes: int, K, C, order,
                                 max_tiles, capacity):
    return _check("smoe_render_workspace_layout",
                  lib.smoe_render_workspace_layout(ct.byref(bins), workspace_ptr, nbytes, K, C,
                                                   order, max_tiles, capacity))


def smoe_bin(model: SmoeModel, grid: SmoeGrid, bins: SmoeBins, stream: int | None):
    return _check("smoe_bin", lib.smoe_bin(ct.byref(model), ct.byref(grid), ct.byref(bins),
                                           stream))


def smoe_render(model, grid, bins, image_ptr, denom_ptr, target_ptr, loss_ptr, stream):
    return _check("smoe_render",
                  lib.smoe_render(ct.byref(model), ct.byref(grid), ct.byref(bins), image_ptr,
                                  denom_ptr, target_ptr, loss_ptr, stream))


def smoe_render_backward(model, grid, bins, image_ptr, denom_ptr, grad_image_ptr, target_ptr,
                         grads_ptr, stream):
    return _check("smoe_render_backward",
                  lib.smoe_render_backward(ct.byref(model), ct.byref(grid), ct.byref(bins),
                                           image_ptr, denom_ptr, grad_image_ptr, target_ptr,
                                           grads_ptr, stream))


def smoe_materialize(K, C, order, raw_ptr, model_ptr, stream):
    return _check("smoe_materialize", lib.smoe_materialize(K, C, order, raw_ptr, model_ptr,
                                                           stream))


def smoe_fit_step(state: SmoeFitState, target_ptr, loss_ptr, stream):
    return _check("smoe_fit_step", lib.smoe_fit_step(ct.byref(state), target_ptr, loss_ptr,
                                                     stream))


def smoe_fit_step_timed(state: SmoeFitState, target_ptr, loss_ptr, events4, stream):
    """events4: four hipEvent_t handles (ints) or None entries."""
    arr = (_vp * 4)(*[e or None for e in events4])
    return _check("smoe_fit_step_timed",
                  lib.smoe_fit_step_timed(ct.byref(state), target_ptr, loss_ptr, arr, stream))


def smoe_pair_stats(model, grid, bins, out2_ptr, stream):
    return _check("smoe_pair_stats", lib.smoe_pair_stats(ct.byref(model), ct.byref(grid),
                                                         ct.byref(bins), out2_ptr, stream))


def smoe_read_status(bins: SmoeBins, stream):
    """Returns (code, [P needed, overflow, longest list, non-finite flag]); code may be
    CAPACITY or NONFINITE."""
    out = (_i32 * 4)()
    code = _check("smoe_read_status", lib.smoe_read_status(ct.byref(bins), out, stream),
                  allow=(SMOE_ERR_CAPACITY, SMOE_ERR_NONFINITE))
    return code, list(out)


def smoe_segments_layout(segs):
    """segs: ctypes array of SmoeSegment, filled in place; returns (K, T, pixels)."""
    k, t, px = _i32(), _i32(), ct.c_int64()
    _check("smoe_segments_layout", lib.smoe_segments_layout(segs, len(segs), ct.byref(k),
                                                            ct.byref(t), ct.byref(px)))
    return k.value, t.value, px.value


def smoe_bin_batched(batch: SmoeBatch, bins: SmoeBins, stream):
    return _check("smoe_bin_batched", lib.smoe_bin_batched(ct.byref(batch), ct.byref(bins), stream))


def smoe_render_batched(batch: SmoeBatch, bins: SmoeBins, images_ptr, denoms_ptr, stream):
    return _check("smoe_render_batched", lib.smoe_render_batched(ct.byref(batch), ct.byref(bins),
                                                                 images_ptr, denoms_ptr, stream))


def smoe_fit_segment_losses(state: SmoeFitState, out_ptr, stream):
    return _check("smoe_fit_segment_losses", lib.smoe_fit_segment_losses(ct.byref(state), out_ptr,
                                                                         stream))


def smoe_render_noalloc(model, grid, image_ptr, denom_ptr, status_ptr, stream):
    return _check("smoe_render_noalloc",
                  lib.smoe_render_noalloc(ct.byref(model), ct.byref(grid), image_ptr, denom_ptr,
                                          status_ptr, stream))


def smoe_fuse_windows(windows_ptr, C_, width, height, window, displacement, image_ptr, stream):
    return _check("smoe_fuse_windows",
                  lib.smoe_fuse_windows(windows_ptr, C_, width, height, window, displacement,
                                        image_ptr, stream))


def smoe_issue_probe(kind, iters, workgroups, out_ptr, stream):
    return _check("smoe_issue_probe", lib.smoe_issue_probe(kind, iters, workgroups, out_ptr, stream))
