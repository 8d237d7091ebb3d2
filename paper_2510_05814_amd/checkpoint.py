"""Model files and fit checkpoints.

Both are safetensors files: named tensors plus string metadata, which a load only parses --
nothing in a file is executed.

save_model / load_model: one fitted model -- its raw rows [K, 6 + C(1 + 2 order)] (mu_x,
mu_y, s1, l21, s2, rho, then the experts), with C, the expert order, the native raster size
and the rule's settings (radius, box, mode, reading of the truncation).  A server loads such
files into a ModelBank (serve.py) instead of fitting in-process.

save_fit / resume_fit: a single-image fit in progress -- raw rows, Adam's moments m and v,
the device step counter, the loss history and the Adam settings.  The resumed state
re-derives the block rectangles and render records from the rows exactly as the
uninterrupted fit's Adam step does, so it continues bit for bit as if never stopped.
"""
from __future__ import annotations

import dataclasses
import json

import torch
from safetensors.torch import load_file, save_file

from .core import AdamConfig, FitState, materialize, num_params

FORMAT_MODEL = "smoe-model-1"
FORMAT_FIT = "smoe-fit-1"


def _meta_common(C_: int, order: int, width: int, height: int, radius: float, box: str,
                 mode: str, trunc: str) -> dict:
    return {"C": str(int(C_)), "order": str(int(order)), "width": str(int(width)),
            "height": str(int(height)), "radius": repr(float(radius)), "box": str(box),
            "mode": str(mode), "trunc": str(trunc)}


def _check_rows(raw: torch.Tensor, C_: int, order: int):
    if raw.dtype != torch.float32 or raw.dim() != 2 or raw.shape[1] != num_params(C_, order):
        raise ValueError(f"raw rows must be float32 [K, {num_params(C_, order)}]")


def save_model(path: str, raw: torch.Tensor, C_: int, order: int, width: int, height: int,
               radius: float = 3.0, box: str = "square", mode: str = "smoe",
               trunc: str = "gradient"):
    """Writes one model's raw rows and settings to `path`."""
    raw = raw.detach().to("cpu").contiguous()
    _check_rows(raw, C_, order)
    meta = {"format": FORMAT_MODEL, **_meta_common(C_, order, width, height, radius, box, mode,
                                                  trunc)}
    save_file({"raw": raw}, path, metadata=meta)


def _read(path: str, fmt: str):
    from safetensors import safe_open

    with safe_open(path, framework="pt") as f:
        meta = f.metadata() or {}
    if meta.get("format") != fmt:
        raise ValueError(f"{path}: not a {fmt} file (format {meta.get('format')!r})")
    return load_file(path), meta


def load_model(path: str, device="cpu"):
    """(raw rows [K, NP] on `device`, info dict: C, order, width, height, radius, box, mode,
    trunc) of a file written by save_model."""
    t, meta = _read(path, FORMAT_MODEL)
    info = {"C": int(meta["C"]), "order": int(meta["order"]), "width": int(meta["width"]),
            "height": int(meta["height"]), "radius": float(meta["radius"]), "box": meta["box"],
            "mode": meta["mode"], "trunc": meta["trunc"]}
    raw = t["raw"]
    _check_rows(raw, info["C"], info["order"])
    return raw.to(device), info


def load_models_materialized(paths, device="cuda"):
    """Materialized rows of each model file (for a ModelBank) and their infos."""
    rows, infos = [], []
    for p in paths:
        raw, info = load_model(p, device)
        rows.append(materialize(raw.contiguous(), info["C"], info["order"]))
        infos.append(info)
    return rows, infos


def save_fit(path: str, st: FitState):
    """Checkpoint of a single-image fit: rows, moments, step counter, loss history, settings."""
    if st.batched:
        raise ValueError("checkpoints cover single-image fits")
    torch.cuda.synchronize()
    tensors = {"raw": st.raw.cpu(), "m": st.m.cpu(), "v": st.v.cpu(),
               "step": st.step_counter.cpu(), "loss_history": st.loss_history.cpu()}
    g = st.grid
    meta = {"format": FORMAT_FIT,
            **_meta_common(st.C, st.order, st.W, st.H, g.radius, st.box, st.mode, st.trunc),
            "adam": json.dumps(dataclasses.asdict(st.adam)), "max_steps": str(st.max_steps),
            "write_render": str(int(st.write_render))}
    save_file(tensors, path, metadata=meta)


def resume_fit(path: str, target: torch.Tensor, capacity: int | None = None) -> FitState:
    """A FitState for `target` continuing the checkpointed fit at its next step."""
    t, meta = _read(path, FORMAT_FIT)
    C_, order = int(meta["C"]), int(meta["order"])
    if tuple(target.shape) != (int(meta["height"]), int(meta["width"]), C_):
        raise ValueError("the target does not match the checkpoint's raster")
    dev = target.device
    st = FitState(target, t["raw"].to(dev), order, AdamConfig(**json.loads(meta["adam"])),
                  max_steps=int(meta["max_steps"]), capacity=capacity,
                  radius=float(meta["radius"]), box=meta["box"], mode=meta["mode"],
                  trunc=meta["trunc"], write_render=bool(int(meta["write_render"])))
    st.m.copy_(t["m"].to(dev))
    st.v.copy_(t["v"].to(dev))
    st.step_counter.copy_(t["step"].to(dev))
    n = min(st.loss_history.numel(), t["loss_history"].numel())
    st.loss_history[:n].copy_(t["loss_history"][:n].to(dev))
    torch.cuda.synchronize()
    return st
