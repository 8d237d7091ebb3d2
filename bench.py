#!/usr/bin/env python3
"""Benchmark of the rasterized SMoE fit step on one MI355X.

Workload: fit of a 2048x2048 RGB float32 denoising target (Voronoi ramps + Gaussian noise
of std 25/255) with K = 65536 linear-expert kernels initialised on a 256x256 grid
(sigma 4 px), truncation radius 3, 16x16 blocks, Adam with the paper's learning rates.
A step is one full iteration of the hot path: binning (box, block lists, ordering),
forward render with the fused loss, backward, and the fused gradient-reduce/Adam/
re-materialize update -- one smoe_fit_step call; most timed steps replay from HIP graphs
captured beforehand.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  Besides throughput it reports the roofline of the dominant kernel
(its duration from HIP events recorded around it in every timed step), the oracle's CPU
throughput on a bounded sample of the same workload, per-stage times and pair counts.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20]
    python bench.py --summarize-profile DIR   # writes profiles/ summaries of rocprofv3 runs
"""
from __future__ import annotations

import argparse
import ctypes as ct
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SMoE fit iters/s (fwd+bwd) 2048² K=65536; render p50/p99 latency vs plain"
WORKLOAD = "fit-2048x2048-rgb-K65536-linear-denoise"

# Algorithmic FP32 work per (pixel, kernel) pair, in VALU operations (one add, mul, fma,
# compare or exp each), C = 3 linear experts, counted on the plain per-pair formulas (not on
# this implementation, which shares column terms between a lane's pixels):
#   tested pair (the truncation test):  dx, dy, z1, l21*z1, w, z2, z1^2, z2^2, q, compare = 10
#   forward, every tested pair: exponent fma, exp, D add, 6 fma expert, 3 fma numerators = 12
#   backward, pair inside the ellipse: exponent fma, exp, w = e/D, 6 expert fma, 3 G fma,
#     H = w G, drho += H, 3 g w products and 3 da adds, 6 dW fma, bz2, 2 bz1, 2 x 4 for
#     bdx / bdy (1/l, 3 slope fma), 2 dmu, ds1 fma, 2 dl21, ds2 fma = 43, rounded up to the
#     45 of the hot-path survey
OPS_TESTED = 10
OPS_ACTIVE_FWD = 12
OPS_ACTIVE_BWD = 45
# MI355X FP32 vector peak: 157.3 TFLOP/s counting an FMA as 2 flops = 256 CUs x 4 SIMDs x
# 32 lanes x 2.4 GHz = 78.6e12 lane-operations/s (one FP32 instruction per lane).  The
# counters agree: the fused kernel issues more than one wave64 VALU instruction per 4 cycles
# per SIMD, so a wave64 FP32 instruction takes 2 cycles without packed math.
VALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
HBM_PEAK = 8.0e12

STAGES = ["bin", "render_backward", "adam"]
DOMINANT = "render_backward"
KERNEL_NAMES = {"render_backward": "k_fit_tile"}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_fit2048.json")
CALIB_BYTES = 1 << 30


# ----------------------------------------------------------------------------- HIP events

class HipEvents:
    """hipEventCreate/ElapsedTime through the HIP runtime torch already loaded."""

    def __init__(self):
        self.lib = ct.CDLL("libamdhip64.so.7")
        self.lib.hipEventCreate.argtypes = [ct.POINTER(ct.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ct.POINTER(ct.c_float), ct.c_void_p, ct.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ct.c_void_p]
        self.lib.hipEventSynchronize.argtypes = [ct.c_void_p]

    def create(self, n):
        out = []
        for _ in range(n):
            e = ct.c_void_p()
            if self.lib.hipEventCreate(ct.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            out.append(e.value)
        return out

    def elapsed_ms(self, a, b):
        self.lib.hipEventSynchronize(b)
        f = ct.c_float()
        if self.lib.hipEventElapsedTime(ct.byref(f), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(f.value)

    def record(self, e, stream_handle):
        if self.lib.hipEventRecord(ct.c_void_p(e), ct.c_void_p(stream_handle)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def destroy(self, evs):
        for e in evs:
            self.lib.hipEventDestroy(e)


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "render_backward": ["paper_2510_05814_amd/csrc/fit.hip", "paper_2510_05814_amd/csrc/tile_math.h",
                        "paper_2510_05814_amd/csrc/device_common.h",
                        "paper_2510_05814_amd/csrc/smoe_internal.h"],
}


# ----------------------------------------------------------------------------- CPU baseline

def cpu_baseline(target, raw0, budget_s=20.0):
    """The FP64 oracle's loss + gradient on a band of image rows with all K kernels, scaled
    to iterations/s of the whole 2048^2 image.  Every pixel of the band visits all K kernels
    (the oracle's plain definition), exactly as a full-image call would."""
    import numpy as np

    import oracle

    H, W, C = target.shape
    threads = oracle.default_threads()
    model = oracle.materialize(raw0.astype(np.float64), C, 1)
    # grow the band until one call takes about budget_s (at most three resizes)
    rows = 8
    for _ in range(4):
        t0 = time.perf_counter()
        oracle.loss_grad(model, C, 1, W, rows, target=target[:rows], threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * budget_s or rows >= H:
            break
        rows = int(min(H, max(rows + 8, rows * 0.9 * budget_s / max(dt, 1e-3))))
        rows -= rows % 8
    full_s = dt * H / rows
    out = {"value": 1.0 / full_s, "unit": "iters/s", "cores": threads, "kind": "oracle",
           "sample": f"FP64 loss+gradient over rows 0..{rows - 1} ({W}x{rows} px) with all "
                     f"{raw0.shape[0]} kernels, {dt:.1f} s, scaled by {H}/{rows} rows",
           "seconds_per_iter": full_s}
    # the small fit workload, whole: 64^2 grey, K = 64 constant experts, 100 Adam steps at 1e-2
    import workloads as wl
    w1 = wl.workload(1)
    t0 = time.perf_counter()
    hist, _ = oracle.fit(w1.raw0.astype(np.float64), 1, 0, w1.target, 100, threads=threads)
    dt1 = time.perf_counter() - t0
    out["fit_64x64_K64_100_steps"] = {"seconds": dt1, "iters_per_s": 100.0 / dt1,
                                      "final_loss": float(hist[-1])}
    return out


# ----------------------------------------------------------------------------- main bench

_T0 = time.perf_counter()


def run(args):
    import numpy as np
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi
    import workloads as wl

    torch.cuda.set_device(0)
    w = wl.workload(3)
    H, W, C = w.target.shape
    target = torch.from_numpy(w.target).cuda()
    clean = torch.from_numpy(w.clean).cuda()
    adam = smoe.AdamConfig(total_steps=10000)
    raw0 = torch.from_numpy(w.raw0).cuda()
    b0 = smoe.bin(smoe.materialize(raw0, C, 1), C, 1, smoe.make_grid(W, H))
    P0 = b0.read_status()[1][0]
    del b0
    # The fit state's own bucket width: twice the initial longest list, at least 64 (the
    # lists of this fit stay below 50 entries, so every block's list is one chunk and the
    # single-chunk fit kernel runs; an overflowed step would be a no-op and is checked below).
    # The timed steps need only the loss, the gradient and the update: the render is not
    # stored (write_render off); the PSNR below comes from a render of the model afterwards.
    st = smoe.FitState(target, raw0, 1, adam,
                       max_steps=args.prefit + args.warmup + args.steps + 16,
                       write_render=False)
    ev = HipEvents()
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    # The window is timed late in the fit: the block lists grow from the initial geometry
    # (P = 260 100) over the first few hundred steps and then stay long, so steps after the
    # pre-fit are the ones a fit spends most of its time in.  Pre-fit steps replay from
    # graphs; then warm-up steps, then a check that the pair capacity is sufficient.
    if args.prefit:
        st.run_graphed(args.prefit)
    for _ in range(args.warmup):
        st.step()
    st.grow_if_needed()

    # per-stage profile of a few steps (not part of the timed region)
    nprof = 8
    ne = len(STAGES) + 1
    evs = ev.create(ne * nprof)
    for i in range(nprof):
        st.step_timed(evs[ne * i:ne * i + ne])
    torch.cuda.synchronize()
    stage_ms = {s: [] for s in STAGES}
    for i in range(nprof):
        e = evs[ne * i:ne * i + ne]
        for k, s in enumerate(STAGES):
            stage_ms[s].append(ev.elapsed_ms(e[k], e[k + 1]))
    ev.destroy(evs)
    stage_avg = {s: float(np.mean(v)) for s, v in stage_ms.items()}
    dominant = DOMINANT
    dom_idx = STAGES.index(dominant)

    # Timed region: K steps.  The first K - M replay from HIP graphs of up to 50 captured
    # steps; the last M run eagerly with HIP events recorded around the dominant kernel on
    # its launch stream (HIP does not time events recorded as graph nodes), which gives the
    # kernel's average launch duration from inside the timed region.
    m_ev = max(1, min(20, args.steps // 5))
    n_graph = 0 if args.eager else args.steps - m_ev
    m_ev = args.steps - n_graph
    spg = max(1, min(n_graph, 50))
    n_full, rem = divmod(n_graph, spg) if n_graph > 0 else (0, 0)
    graph = st.capture(spg) if n_full else None
    graph_rem = st.capture(rem) if rem else None
    evs = ev.create(2 * m_ev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_full):
        st.replay(graph)
    if graph_rem is not None:
        st.replay(graph_rem)
    for i in range(m_ev):
        e4 = [None] * ne
        e4[dom_idx], e4[dom_idx + 1] = evs[2 * i], evs[2 * i + 1]
        st.step_timed(e4)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms = [ev.elapsed_ms(evs[2 * i], evs[2 * i + 1]) for i in range(m_ev)]
    ev.destroy(evs)
    elapsed = t1 - t0
    over, status = st.bins.read_status()
    if over:
        raise RuntimeError("pair capacity overflow inside the timed region")

    # geometry at the end of the timed region, from a standalone binning of the current model
    # (the fit workspace already holds part of the next step's binning)
    sb = smoe.bin(st.model, C, 1, st.grid)
    _, sstat = sb.read_status()
    stats = torch.zeros(2, dtype=torch.int64, device="cuda")
    m = smoe.core.model_struct(st.model, C, 1)
    _capi.smoe_pair_stats(m, st.grid, sb.c, stats.data_ptr(), sh)
    tested, active = [int(x) for x in stats.tolist()]
    P = sstat[0]
    status = sstat
    T = smoe.tiles(W, H)

    dom_avg_s = float(np.mean(dom_ms)) * 1e-3
    # the fused kernel tests every pair twice (forward, then the recomputing backward); the
    # forward accumulates every tested pair (the block lists decide the render, Sec. IV-B),
    # the backward only the pairs inside the ellipse
    ops = tested * (2 * OPS_TESTED + OPS_ACTIVE_FWD) + active * OPS_ACTIVE_BWD
    achieved = ops / dom_avg_s
    roofline = {"bound": "alu", "kernel": KERNEL_NAMES[dominant], "achieved": achieved / 1e12,
                "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s (FP32 VALU lane-ops)",
                "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                "avg_launch_ms": dom_avg_s * 1e3, "algorithmic_ops_per_launch": ops,
                "duration_source": f"HIP events around the kernel in the last {m_ev} timed "
                                   f"steps (eager); the other {n_graph} replay from graphs"}
    # HBM traffic per launch from committed rocprofv3 counters, if taken on this source
    try:
        with open(COUNTERS_FILE) as f:
            k = json.load(f)["kernels"][KERNEL_NAMES[dominant]]
        if k["source_digest"] == source_digest(KERNEL_SOURCES[dominant]):
            roofline["traffic"] = k["fetch_bytes"] + k["write_bytes"]
    except (OSError, ValueError, KeyError):
        pass

    img_now, _, _, _ = smoe.render(st.model, C, 1, st.grid)
    psnr_clean = smoe.psnr(img_now, clean)
    steps_before = args.prefit + args.warmup + nprof
    out = {
        "metric": METRIC, "value": args.steps / elapsed, "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "image": f"{W}x{H}x{C}", "K": st.K, "experts": "linear",
                   "tile": 16, "radius": 3.0, "fit_steps_before_timing": steps_before,
                   "timed_steps": [steps_before, steps_before + args.steps],
                   "truncation": "block lists in the render, ellipse in the gradient",
                   "render_stored_per_step": False},
        "roofline": roofline,
        "stages_ms": stage_avg,
        "pairs": {"P_init": P0, "P": P, "mean_list": P / T, "longest_list": status[2], "tested": tested,
                  "active": active, "active_per_px": active / (W * H)},
        "gate_evals_per_s_tested": tested * args.steps / elapsed,
        "psnr_vs_clean_db": psnr_clean,
        "cpu_baseline": None,
    }
    _progress(f"headline {out['value']:.1f} it/s")
    out["bin_render"] = run_bin_render(st, C)
    if not args.no_early_window:
        out["early_window"] = run_early_window(args, w, P0)
        _progress("early_window")
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w.target, w.raw0, budget_s=args.cpu_budget)
        out["cpu_baseline"] = cb
        _progress("cpu_baseline")
    if not args.no_serving:
        out["serving"] = run_serving(args)
        _progress("serving")
    if not args.no_batched_fit:
        out["batched_fit"] = run_batched_fit(args)
        _progress("batched_fit")
    if not args.no_mm:
        out["mm_denoise"] = run_mm_denoise(args)
        _progress("mm_denoise")
    if not args.no_tight:
        out["tight_box"] = run_tight_box(args)
        _progress("tight_box")
    if not args.no_rbf:
        out["rbf_vs_smoe"] = run_rbf_vs_smoe(args)
        _progress("rbf_vs_smoe")
    if not args.no_long:
        out["long_lists"] = run_long_lists(args)
        _progress("long_lists")
    if not args.no_readings:
        out["truncation_readings"] = run_truncation_readings(args)
        _progress("truncation_readings")
    if not args.no_small:
        out["small_fits"] = run_small_fits(args)
        _progress("small_fits")
    if not args.no_autograd:
        out["autograd"] = run_autograd(args, w)
        _progress("autograd")
    if not args.no_peaks:
        out["peaks"] = run_peaks()
        _progress("peaks")
    if not args.no_trunc_report:
        out["truncation_error"] = truncation_report(w)
        _progress("truncation_error")
    if args.copy_calibration:
        # One-dispatch streaming kernel of known size (reads and writes CALIB_BYTES each),
        # for scaling the FETCH_SIZE / WRITE_SIZE counters.  Sized above the 256 MB MALL.
        a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = CALIB_BYTES
    print(json.dumps(out), flush=True)


def _progress(what):
    """One line on stderr per finished section (the JSON result goes to stdout)."""
    print(f"[bench] {what} done at {time.perf_counter() - _T0:.0f} s", file=sys.stderr, flush=True)


def run_bin_render(st, C):
    """The standalone calls a served full-image request makes -- smoe_bin (box, block
    counts, scan, scatter, per-block sort) and smoe_render -- on the headline model at the end
    of the timed window, into preallocated buffers, with HIP events recorded on the calls'
    stream around each; medians over 50 iterations after 5 warm-up ones."""
    import numpy as np
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi

    b = smoe.bin(st.model, C, 1, st.grid)
    _, stat = b.read_status()
    H, W = st.grid.height, st.grid.width
    img = torch.empty((H, W, C), dtype=torch.float32, device="cuda")
    den = torch.empty((H, W), dtype=torch.float32, device="cuda")
    m = smoe.core.model_struct(st.model, C, 1)
    sh = torch.cuda.current_stream().cuda_stream
    ev = HipEvents()
    n = 50
    evs = ev.create(3 * n)
    for i in range(-5, n):
        if i >= 0:
            ev.record(evs[3 * i], sh)
        _capi.smoe_bin(m, st.grid, b.c, sh)
        if i >= 0:
            ev.record(evs[3 * i + 1], sh)
        _capi.smoe_render(m, st.grid, b.c, img.data_ptr(), den.data_ptr(), None, None, sh)
        if i >= 0:
            ev.record(evs[3 * i + 2], sh)
    torch.cuda.synchronize()
    t_bin = [ev.elapsed_ms(evs[3 * i], evs[3 * i + 1]) for i in range(n)]
    t_ren = [ev.elapsed_ms(evs[3 * i + 1], evs[3 * i + 2]) for i in range(n)]
    ev.destroy(evs)
    over, _ = b.read_status()
    if over:
        raise RuntimeError("standalone binning overflowed its workspace")
    return {"bin_ms": float(np.median(t_bin)), "render_ms": float(np.median(t_ren)),
            "P": int(stat[0]), "longest_list": int(stat[2]), "iterations": n}


def run_peaks():
    """Measured ceilings beside the published peaks.  The issue-rate probe (smoe_issue_probe):
    8 waves per SIMD on all 1024 SIMDs, each lane running 8 independent chains of one FP32
    instruction -- fma on vector registers, fma reading a scalar register, v_exp_f32 -- timed
    with events on the launch's stream; and a 1 GiB device-to-device copy (HBM read + write)."""
    import torch

    from paper_2510_05814_amd import _capi

    sh = torch.cuda.current_stream().cuda_stream
    wg = 1024 * 8 // 4                      # 256-thread workgroups: 4 waves each
    out = torch.empty(wg * 256, dtype=torch.float32, device="cuda")
    res = {"waves_per_simd": 8, "chains_per_lane": 8}
    for kind, name in ((0, "fma_vector"), (1, "fma_scalar_operand"), (2, "exp")):
        iters = 2048
        _capi.smoe_issue_probe(kind, 64, wg, out.data_ptr(), sh)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _capi.smoe_issue_probe(kind, iters, wg, out.data_ptr(), sh)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        instr = wg * 4 * iters * 8
        r = {"ms": t * 1e3, "wave_instr_per_simd_cycle_at_2.4GHz": instr / (N_SIMD * CLOCK_HZ * t),
             "of_published_rate": instr / (N_SIMD * CLOCK_HZ * t) / 0.5}
        if kind < 2:
            r["tflops"] = instr * 64 * 2 / t / 1e12
        res[name] = r
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / 5
    res["hbm_copy_gbps"] = 2 * a.numel() * 4 / t / 1e9
    res["hbm_copy_of_peak"] = res["hbm_copy_gbps"] * 1e9 / HBM_PEAK
    del a, b
    torch.cuda.empty_cache()
    return res


def run_small_fits(args):
    """The two smaller fit workloads, each fitted for its full length: 64^2 grey with K = 64
    constant experts for 100 Adam steps (lr 1e-2; launch-bound), and 512^2 RGB with K = 4096
    linear experts for 2000 steps (the paper's rates).  Iterations/s over the whole fit (after
    the first, eager step) and the final PSNR against the target."""
    import torch

    import paper_2510_05814_amd as smoe
    import workloads as wl

    out = {}
    for n, adam in ((1, smoe.AdamConfig.constant(1e-2, 100)), (2, None)):
        w = wl.workload(n)
        steps = w.steps
        adam = adam or smoe.AdamConfig(total_steps=steps)
        t = torch.from_numpy(w.target).cuda()
        st = smoe.FitState(t, torch.from_numpy(w.raw0).cuda(), w.order, adam, max_steps=steps)
        st.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.run_graphed(steps - 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        img, _, _, _ = smoe.render(st.model, t.shape[2], w.order, st.grid)
        out[w.name] = {"steps": steps, "iters_per_s": (steps - 1) / dt,
                       "fit_s": dt * steps / (steps - 1), "final_mse": float(st.losses()[-1]),
                       "psnr_db": smoe.psnr(img, t)}
    return out


def run_autograd(args, w):
    """The differentiable render (torch.autograd.Function) on the headline workload: per
    iteration a forward (materialize, bin, render), the MSE to the target in torch, the
    backward through the hand-written adjoint and a torch.optim.Adam step, all eager on one
    stream (autograd is not captured in a graph).  Both readings: the exact adjoint (the
    Function's default) and the fit step's reading.  Iterations/s over the timed steps, after
    warm-up steps from the grid init, beside the fused fit step's rate."""
    import torch

    from paper_2510_05814_amd.autograd import smoe_render

    H, W, C = w.target.shape
    t = torch.from_numpy(w.target).cuda()
    out = {"steps": args.autograd_steps, "warmup": 5, "optimizer": "torch.optim.Adam lr 1e-2"}
    for trunc in ("render", "gradient"):
        r = torch.from_numpy(w.raw0).cuda().requires_grad_(True)
        opt = torch.optim.Adam([r], lr=1e-2)

        def it():
            opt.zero_grad(set_to_none=False)
            loss = torch.mean((smoe_render(r, C, 1, W, H, trunc=trunc) - t) ** 2)
            loss.backward()
            opt.step()
            return loss

        for _ in range(5):
            it()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.autograd_steps):
            loss = it()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[trunc] = {"iters_per_s": args.autograd_steps / dt,
                      "ms_per_iter": 1e3 * dt / args.autograd_steps, "last_loss": loss.item()}
        del r, opt
        torch.cuda.empty_cache()
    return out


def truncation_report(w):
    """Truncation error of the rasterized model (Sec. IV-B) against the global model of
    Sec. III-B (every kernel at every pixel), on a 256^2 crop of the headline workload with
    its K = 1024 kernels at the initial geometry, by the FP64 oracle: the image error of each
    reading and of the uncut block lists against the untruncated render."""
    import numpy as np

    import oracle

    t0 = time.perf_counter()
    gx = 32                                  # 32 x 32 kernels (spacing 8) over 256^2
    raw = w.raw0.reshape(256, 256, -1)[:gx, :gx].reshape(gx * gx, -1).astype(np.float64)
    model = oracle.materialize(raw, 3, 1)
    S = 256
    y_all, _ = oracle.render(model, 3, 1, S, S, truncated=False)
    rows = {}
    for name, kw in (("block_lists_representable", dict(trunc="gradient")),
                     ("ellipse_in_render", dict(trunc="render")),
                     ("block_lists_uncut", dict(truncated="lists"))):
        y, D = oracle.render(model, 3, 1, S, S, **kw)
        d = y - y_all
        rows[name] = {"max_abs": float(np.max(np.abs(d))), "rms": float(np.sqrt(np.mean(d * d))),
                      "psnr_vs_untruncated_db": float(10 * np.log10(1.0 / max(np.mean(d * d), 1e-300))),
                      "uncovered_px": int((D == 0).sum())}
    return {"crop": f"{S}x{S}", "K": int(model.shape[0]), "geometry": "initial (sigma 4, spacing 8)",
            "radius": 3.0, "vs_untruncated": rows, "seconds": time.perf_counter() - t0}


def run_early_window(args, w, P0):
    """The same fit timed early, over steps [20, 220) from the initial geometry (shorter block
    lists than later in the fit), all steps replayed from graphs: context for the headline."""
    import torch

    import paper_2510_05814_amd as smoe

    target = torch.from_numpy(w.target).cuda()
    st = smoe.FitState(target, torch.from_numpy(w.raw0).cuda(), 1,
                       smoe.AdamConfig(total_steps=10000), max_steps=256, write_render=False)
    for _ in range(20):
        st.step()
    st.grow_if_needed()
    g = st.capture(50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        st.replay(g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if st.bins.read_status()[0]:
        raise RuntimeError("pair capacity overflow in the early window")
    return {"timed_steps": [20, 220], "iters_per_s": 200 / dt, "ms_per_step": 1e3 * dt / 200}


# ----------------------------------------------------------------------------- serving

def run_serving(args):
    """Serving workload: 16 resident fitted models (K 256 .. 65536, native 256^2 .. 2048^2,
    linear experts), a Poisson stream of render requests at 200 req/s, each at an upscale
    factor in {1, 2, 3, 4} with outputs up to 4096^2 RGB, admitted under an 8 GB budget.
    Reports p50/p99 latency and pixels/s of continuous batching against one launch
    sequence per request, at the Poisson rate, at saturation (all requests at t = 0), and at
    higher Poisson rates (2000, 5000, 10000 req/s) of the same request mix."""
    import numpy as np
    import torch

    import tempfile

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import checkpoint as ck
    from paper_2510_05814_amd.serve import ModelBank, PlainServer, Server
    import workloads as wl

    t_setup = time.perf_counter()
    ms = wl.serving_models()
    st = smoe.FitState([torch.from_numpy(m["image"]).cuda() for m in ms],
                       [torch.from_numpy(m["raw0"]).cuda() for m in ms], 1,
                       smoe.AdamConfig(total_steps=args.serve_fit_steps),
                       max_steps=args.serve_fit_steps)
    for _ in range(args.serve_fit_steps):
        st.step()
    st.grow_if_needed()
    # the server loads the fitted models from model files, as a deployment would
    with tempfile.TemporaryDirectory() as td:
        paths = []
        for i, (sg, m) in enumerate(zip(st.segments.host, ms)):
            paths.append(os.path.join(td, f"model{i}.safetensors"))
            ck.save_model(paths[-1], st.raw[sg.kernel_offset:sg.kernel_offset + sg.num_kernels],
                          3, 1, m["side"], m["side"])
        models, _ = ck.load_models_materialized(paths)
    bank = ModelBank(models, 3, 1)
    del st
    torch.cuda.empty_cache()
    sides = [m["side"] for m in ms]
    reqs = wl.serving_requests(sides, args.serve_requests, rate=200.0)
    warm = wl.serving_requests(sides, 24, rate=1e6, seed=7)
    setup_s = time.perf_counter() - t_setup
    out = {"models": len(ms), "K": [m["K"] for m in ms], "native_side": sides,
           "requests": len(reqs), "rate_hz": 200.0, "scales": [1, 2, 3, 4], "max_side": 4096,
           "budget_bytes": 8 << 30, "mean_output_px": float(np.mean([r["width"] * r["height"]
                                                                    for r in reqs])),
           "setup_s": setup_s, "fit_steps_per_model": args.serve_fit_steps}
    srv = Server(bank, budget_bytes=8 << 30, streams=2, overlap_backlog=args.serve_overlap_backlog,
                 fill_blocks=args.serve_fill_blocks, reserve_for=(4096, 4096, (1, 2, 3, 4)))
    plain = PlainServer(bank)
    # warm-up, the same for both servers: the largest window of every model at every scale
    # (so that the allocator's cache holds blocks of every output and workspace size), then a
    # random mix
    largest = [dict(model=i, scale=sc, width=min(4096, sides[i] * sc),
                    height=min(4096, sides[i] * sc), arrival=0.0)
               for i in range(len(sides)) for sc in (1, 2, 3, 4)]
    for wq in (largest, warm):
        srv.serve(wq, realtime=False)
        plain.serve(wq, realtime=False)
        srv.serve(wq, realtime=True)
        plain.serve(wq, realtime=True)
    # The two servers on the same request stream, in the order batched, plain, plain,
    # batched, so that a drift of the GPU's clocks or of the host over the section lands on
    # both alike; each server's two runs are pooled for the latency percentiles (the
    # throughput fields are those of its first run).
    runs = {"batched": [], "plain": []}
    for name, server in (("batched", srv), ("plain", plain), ("plain", plain), ("batched", srv)):
        runs[name].append(server.serve(reqs))
    for name, rs in runs.items():
        summ = dict(rs[0][1])
        res = [r for run, _ in rs for r in run]
        lat = np.array([r.latency for r in res]) * 1e3
        wait = np.array([r.started - r.request.arrival for r in res]) * 1e3
        gpu = np.array([r.done - r.started for r in res]) * 1e3
        summ.update({"runs": len(rs), "order": "batched, plain, plain, batched",
                     "latencies_pooled": len(lat), "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                     "max_ms": float(lat.max()),
                     "wait_p50_ms": float(np.percentile(wait, 50)),
                     "wait_p99_ms": float(np.percentile(wait, 99)),
                     "gpu_p50_ms": float(np.percentile(gpu, 50)),
                     "gpu_p99_ms": float(np.percentile(gpu, 99))})
        out[name] = summ
    # The same rate over independent request streams, which server goes first alternating
    # from stream to stream, latencies pooled: the 99th percentile of one 1000-request run
    # rests on its 10 slowest requests.
    pooled = {"batched": [], "plain": []}
    for rep in range(args.serve_repeats):
        rq = wl.serving_requests(sides, args.serve_requests, rate=200.0, seed=300 + rep)
        pair = (("batched", srv), ("plain", plain))
        for name, server in (pair if rep % 2 == 0 else pair[::-1]):
            res, _ = server.serve(rq)
            pooled[name] += [r.latency * 1e3 for r in res]
    out["pooled_200hz"] = {"streams": args.serve_repeats, "requests_each": args.serve_requests}
    for name, lat in pooled.items():
        if lat:
            out["pooled_200hz"][name] = {"p50_ms": float(np.percentile(lat, 50)),
                                         "p99_ms": float(np.percentile(lat, 99)),
                                         "mean_ms": float(np.mean(lat)), "n": len(lat)}
    if args.serve_one_stream:
        _, out["batched_one_stream"] = Server(bank, budget_bytes=8 << 30, streams=1).serve(reqs)
    sat = reqs[:args.serve_saturation]
    _, out["batched_saturated"] = srv.serve(sat, realtime=False)
    _, out["plain_saturated"] = plain.serve(sat, realtime=False)
    # higher offered loads (same request mix): where batching starts to pay
    out["load_sweep"] = []
    for rate in (2000.0, 5000.0, 10000.0):
        rq = wl.serving_requests(sides, args.serve_sweep_requests, rate=rate, seed=11)
        _, b = srv.serve(rq)
        _, p = plain.serve(rq)
        keys = ("p50_ms", "p99_ms", "pixels_per_s", "requests_per_s")
        out["load_sweep"].append({"rate_hz": rate, "batched": {k: b[k] for k in keys + ("mean_batch",)},
                                  "plain": {k: p[k] for k in keys}})
    return out


def run_batched_fit(args):
    """Batched fit: 64 RGB images of uneven sizes (sides log-uniform in [128, 1024]), each
    with K = pixels / 64 linear experts, fitted together -- one binning + render + backward
    + Adam launch sequence per step for all images, steps replayed from a HIP graph.
    Reports aggregate iterations/s and every image's PSNR against its own unbatched fit
    (the same steps run image by image)."""
    import numpy as np
    import torch

    import paper_2510_05814_amd as smoe
    import workloads as wl

    imgs = wl.config5_images()
    raws = wl.batched_fit_inits(imgs)
    steps = args.bfit_steps
    adam = smoe.AdamConfig(total_steps=steps)
    tg = [torch.from_numpy(i).cuda() for i in imgs]
    rg = [torch.from_numpy(r).cuda() for r in raws]
    probe = smoe.FitState(tg, rg, 1, adam, max_steps=1)
    cap = 2 * probe.bins.capacity        # graph replays cannot re-size the workspace
    del probe
    st = smoe.FitState(tg, rg, 1, adam, max_steps=steps + 1, capacity=cap)
    st.step()                     # first step eagerly (prologue), then graphs
    spg = 50
    n_full, rem = divmod(steps - 1, spg)
    g = st.capture(spg) if n_full else None
    g_rem = st.capture(rem) if rem else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_full):
        st.replay(g)
    if g_rem is not None:
        st.replay(g_rem)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if st.bins.read_status()[0]:
        raise RuntimeError("pair capacity overflow in the batched fit")
    psnr_b = [smoe.psnr(im, t) for im, t in zip(st.images(), tg)]
    # the unbatched path: every image fitted alone for the same steps, its steps replayed
    # from graphs as well (first step eager), timed the same way (graph replays only)
    psnr_u = []
    t_unb = 0.0
    for t, r in zip(tg, raws):
        s1 = smoe.FitState(t, torch.from_numpy(r).cuda(), 1, adam, max_steps=steps + 1)
        s1.step()
        g1 = s1.capture(spg) if n_full else None
        g1_rem = s1.capture(rem) if rem else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_full):
            s1.replay(g1)
        if g1_rem is not None:
            s1.replay(g1_rem)
        torch.cuda.synchronize()
        t_unb += time.perf_counter() - t0
        if s1.bins.read_status()[0]:
            raise RuntimeError("pair capacity overflow in an unbatched fit")
        psnr_u.append(smoe.psnr(s1.image, t))
        del g1, g1_rem, s1
    d = np.abs(np.array(psnr_b) - np.array(psnr_u))
    px = sum(i.shape[0] * i.shape[1] for i in imgs)
    return {"images": len(imgs), "pixels": int(px), "K": int(st.K), "steps": steps,
            "timed_steps": steps - 1, "iters_per_s": (steps - 1) / elapsed,
            "ms_per_step": 1e3 * elapsed / (steps - 1),
            "unbatched_iters_per_s": (steps - 1) / t_unb,
            "unbatched_timing": "each image alone, steps 1.. replayed from graphs, summed",
            "psnr_mean_db": float(np.mean(psnr_b)), "psnr_min_db": float(np.min(psnr_b)),
            "psnr_max_abs_diff_vs_unbatched_db": float(d.max())}


def run_tight_box(args):
    """Square vs tight axis-aligned kernel boxes on fitted models: the headline workload is
    fitted for --tight-fit-steps iterations (square boxes; the paper's 10000 by default),
    then, from that model, for each box: its (block, kernel) pairs, the time of one binning +
    render of the 2048^2 image, and fit iterations/s over --tight-steps graphed steps from
    the same state.  With the ellipse test in the render the images are the same with either
    box, bit for bit (checked); with the block lists deciding the render (the default) the
    tight box drops far tails, and the largest pixel difference is reported."""
    import numpy as np
    import torch

    import paper_2510_05814_amd as smoe
    import workloads as wl

    w = wl.workload(3)
    H, W, C = w.target.shape
    target = torch.from_numpy(w.target).cuda()
    raw0 = torch.from_numpy(w.raw0).cuda()
    n_fit, n_time = args.tight_fit_steps, args.tight_steps
    adam = smoe.AdamConfig(total_steps=10000)
    st = smoe.FitState(target, raw0, 1, adam, max_steps=1, capacity=W * H)
    st.run_graphed(n_fit)
    if st.bins.read_status()[0]:
        raise RuntimeError("pair capacity overflow in the tight-box fit")
    raw = st.raw.clone()
    model = st.model.clone()
    psnr_fit = smoe.psnr(st.image, torch.from_numpy(w.clean).cuda())
    del st
    out = {"workload": WORKLOAD, "fit_steps_before": n_fit, "timed_fit_steps": n_time,
           "psnr_vs_clean_after_fit_db": psnr_fit}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    imgs = {}
    for box in ("square", "tight"):
        # images with the ellipse test in the render, where the tight box is exact
        img_r, _, _, _ = smoe.render(model, C, 1, smoe.make_grid(W, H, box=box, trunc="render"))
        imgs[box + "_render"] = img_r
        grid = smoe.make_grid(W, H, box=box)
        bins = smoe.bin(model, C, 1, grid)
        _, stt = bins.read_status()
        out[f"pairs_{box}"] = int(stt[0])
        out[f"longest_list_{box}"] = int(stt[2])
        img = torch.empty((H, W, C), dtype=torch.float32, device="cuda")
        den = torch.empty((H, W), dtype=torch.float32, device="cuda")
        m = smoe.core.model_struct(model, C, 1)
        sh = torch.cuda.current_stream().cuda_stream
        reps = 50
        for i in range(reps + 5):
            if i == 5:
                ev[0].record()
            smoe._capi.smoe_bin(m, grid, bins.c, sh)
            smoe._capi.smoe_render(m, grid, bins.c, img.data_ptr(), den.data_ptr(), None, None,
                                   sh)
        ev[1].record()
        torch.cuda.synchronize()
        out[f"render_ms_{box}"] = ev[0].elapsed_time(ev[1]) / reps
        imgs[box] = img
        # fit steps from the same fitted state
        f = smoe.FitState(target, raw, 1, adam, max_steps=1, capacity=2 * W * H, box=box)
        f.step()
        g = f.capture(50)
        f.replay(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_time // 50):
            f.replay(g)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if f.bins.read_status()[0]:
            raise RuntimeError("pair capacity overflow in the tight-box fit")
        out[f"fit_iters_per_s_{box}"] = 50 * (n_time // 50) / dt
        del f, g, bins
    out["images_equal_ellipse_in_render"] = bool(torch.equal(imgs["square_render"],
                                                             imgs["tight_render"]))
    out["image_max_abs_diff_default_reading"] = float((imgs["square"] - imgs["tight"]).abs().max())
    out["pair_ratio"] = out["pairs_tight"] / max(1, out["pairs_square"])
    out["render_speedup"] = out["render_ms_square"] / out["render_ms_tight"]
    out["fit_speedup"] = out["fit_iters_per_s_tight"] / out["fit_iters_per_s_square"]
    return out


def run_rbf_vs_smoe(args):
    """The RBF-vs-SMoE contrast of Fig. 2 and Table I, on synthetic step edges: a 512^2 RGB
    piecewise-constant image (12 random lines), clean and with Gaussian noise of std 0.05.
    Gated SMoE (Eq. 2-4) and RBF (Eq. 1) models with the same constant-expert kernels on a
    regular grid (K = 256, 1024 and 4096, sigma = half the spacing; the RBF weights start at the
    grid's kernel density so that both start from the same image scale), the same Adam
    settings (the paper's training protocol, Sec. VI-B: 10 000 iterations by default),
    --rbf-steps iterations each; PSNR of the fit against the clean image."""
    import numpy as np
    import torch

    import paper_2510_05814_amd as smoe
    import workloads as wl

    side, steps = 512, args.rbf_steps
    clean = wl.step_edge_image(seed=31, H=side, W=side, C=3, n_lines=12)
    noisy = wl.step_edge_image(seed=31, H=side, W=side, C=3, n_lines=12, noise_std=0.05)
    c = torch.from_numpy(clean).cuda()
    out = {"image": f"{side}x{side}x3 step edges", "steps": steps, "experts": "constant",
           "runs": []}
    for g in (16, 32, 64):
        spacing = side / g
        sigma = spacing / 2
        for name, img in (("clean", clean), ("noisy", noisy)):
            t = torch.from_numpy(img).cuda()
            row = {"K": g * g, "target": name, "psnr_target_db": smoe.psnr(t, c)}
            for mode in ("smoe", "rbf"):
                raw, _ = wl.grid_init(img, g, g, sigma=sigma, order=0)
                if mode == "rbf":
                    raw[:, 5] = np.float32(math.log(spacing * spacing / (2 * math.pi * sigma ** 2)))
                st = smoe.FitState(t, torch.from_numpy(raw).cuda(), 0,
                                   smoe.AdamConfig(total_steps=steps), max_steps=1, mode=mode)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st.run_graphed(steps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                row[f"psnr_{mode}_db"] = smoe.psnr(st.image, c)
                row[f"iters_per_s_{mode}"] = steps / dt
            out["runs"].append(row)
    return out


# The paper's R-SMoE rows of Table I (Kodak 768x512, constant experts, 10 000 Adam
# iterations, NVIDIA RTX A4000): context only -- another GPU and real photographs.
def run_truncation_readings(args):
    """The two readings of where Sec. IV-B's ellipse discard applies, on the headline
    workload fitted for the paper's 10 000 iterations from the same initialisation: the
    block lists deciding the render with the discard in the gradient (the default), and the
    ellipse test in the render too.  PSNR against the clean image and the fraction of pixels
    no kernel reaches (D = 0) along the way, and fit iterations/s."""
    import torch

    import paper_2510_05814_amd as smoe
    import workloads as wl

    w = wl.workload(3)
    H, W, C = w.target.shape
    target = torch.from_numpy(w.target).cuda()
    clean = torch.from_numpy(w.clean).cuda()
    out = {}
    for trunc in ("gradient", "render"):
        st = smoe.FitState(target, torch.from_numpy(w.raw0).cuda(), 1,
                           smoe.AdamConfig(total_steps=10000), max_steps=1, capacity=W * H,
                           trunc=trunc)
        rows, elapsed, done = [], 0.0, 0
        for goal in (1000, 2000, 5000, 10000):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.run_graphed(goal - done)
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            done = goal
            rows.append({"steps": goal, "psnr_vs_clean_db": smoe.psnr(st.image, clean),
                         "stranded_px_frac": float((st.denom == 0).float().mean().item())})
        out[trunc] = {"trace": rows, "iters_per_s": done / elapsed}
        del st
    return out


def run_long_lists(args):
    """Renders of models with very wide kernels (standard deviations 20-40 px), whose block
    lists run to hundreds or thousands of entries: such blocks are split over four waves.
    Reports pairs, the longest list, the blocks with lists over the split threshold and the
    time of one render (binning excluded), averaged over 20 renders."""
    import torch

    import paper_2510_05814_amd as smoe
    import workloads as wl

    out = []
    for side, K in ((256, 2000), (512, 4000)):
        m = torch.from_numpy(wl.random_model(K, 3, 1, side, side, 5, sig_lo=20.0,
                                             sig_hi=40.0)).cuda()
        grid = smoe.make_grid(side, side)
        _, _, _, b = smoe.render(m, 3, 1, grid)
        _, st = b.read_status()
        rg = b.ranges(smoe.tiles(side, side))
        long_blocks = int(((rg[:, 1] - rg[:, 0]) > 128).sum().item())
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for i in range(25):
            if i == 5:
                ev[0].record()
            smoe.render(m, 3, 1, grid, bins=b)
        ev[1].record()
        torch.cuda.synchronize()
        out.append({"side": side, "K": K, "pairs": int(st[0]), "longest_list": int(st[2]),
                    "blocks": smoe.tiles(side, side), "blocks_split": long_blocks,
                    "render_ms": ev[0].elapsed_time(ev[1]) / 20})
    return out


def run_mm_denoise(args):
    """Multi-model fusion for denoising: the block-overlapping window models of a 512^2 RGB
    image from the denoising workload's generator (clean + N(0, (25/255)^2)), fitted together for each
    displacement d in {16, 8, 4, 2} (H = 1, 4, 16, 64 hypotheses per pixel); PSNR of the
    fused estimate against the clean image, and fit iterations/s of the window batch."""
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.multimodel import MultiModelDenoiser
    import workloads as wl

    clean, noisy = wl.config3_images(H=args.mm_size, W=args.mm_size)
    c = torch.from_numpy(clean).float().cuda()
    out = {"size": args.mm_size, "steps": args.mm_steps,
           "psnr_noisy_db": smoe.psnr(torch.from_numpy(noisy).float().cuda(), c), "runs": []}
    for d in (16, 8, 4, 2):
        mm = MultiModelDenoiser(noisy, d, adam=smoe.AdamConfig(total_steps=args.mm_steps),
                                max_steps=args.mm_steps + 1)
        mm.state.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mm.fit(args.mm_steps - 1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["runs"].append({"d": d, "hypotheses": mm.hypotheses, "windows": len(mm.windows),
                            "kernels": int(mm.state.K), "iters_per_s": (args.mm_steps - 1) / el,
                            "psnr_db": smoe.psnr(mm.image(), c)})
        del mm
        torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------------------- profiles

def _rocpd_kernels(db_path):
    """(name, calls, total ns, average ns, percent of kernel time) from a rocprofv3 SQLite output."""
    import sqlite3

    con = sqlite3.connect(db_path)
    try:
        rows = con.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                           "group by name order by sum(duration) desc").fetchall()
    finally:
        con.close()
    total = sum(r[2] for r in rows) or 1
    return [(n, c, t, a, 100.0 * t / total) for n, c, t, a in rows]


def _rocpd_gaps(db_path, names):
    """Idle time between consecutive dispatches of the fit step's kernels (end of one to
    start of the next, in dispatch order): {"prev->next": [ns, ...]}."""
    import sqlite3

    con = sqlite3.connect(db_path)
    try:
        rows = con.execute('select name, start, "end" from kernels order by start').fetchall()
    except sqlite3.Error:
        return {}
    finally:
        con.close()
    short = []
    for name, t0, t1 in rows:
        k = _kernel_base(name) if _kernel_base(name) in names else None
        short.append((k, t0, t1))
    gaps = {}
    for (a, _, a1), (b, b0, _) in zip(short, short[1:]):
        if a and b:
            gaps.setdefault(f"{a}->{b}", []).append(b0 - a1)
    return gaps


def _rocpd_counters(db_path):
    """{(kernel name, counter): [value per dispatch]} of every PMC counter in a rocprofv3
    SQLite output (rows of one dispatch, e.g. per shader-engine instances, are summed)."""
    import sqlite3

    con = sqlite3.connect(db_path)
    acc = {}
    try:
        for name, disp, ctr, val in con.execute(
                "select kernel_name, dispatch_id, counter_name, value from counters_collection"):
            acc[(name, ctr, disp)] = acc.get((name, ctr, disp), 0.0) + float(val)
    finally:
        con.close()
    out = {}
    for (name, ctr, _), v in acc.items():
        out.setdefault((name, ctr), []).append(v)
    return out


# Kernels of the fit step and of the standalone binning + render, with the sources whose
# digest tags their counters.
_BIN_SRC = ["paper_2510_05814_amd/csrc/binning.hip", "paper_2510_05814_amd/csrc/device_common.h"]
STEP_KERNELS = {"k_fit_tile": KERNEL_SOURCES["render_backward"],
                "k_adam_fit": KERNEL_SOURCES["render_backward"],
                "k_scatter_fixed": _BIN_SRC,
                "k_fill_counts": _BIN_SRC, "k_preprocess": _BIN_SRC, "k_scan": _BIN_SRC,
                "k_scatter": _BIN_SRC, "k_sort_buckets": _BIN_SRC,
                "k_render": ["paper_2510_05814_amd/csrc/render.hip",
                             "paper_2510_05814_amd/csrc/tile_math.h",
                             "paper_2510_05814_amd/csrc/device_common.h"]}


def _kernel_base(name):
    """'void smoe::(anonymous namespace)::k_render<3, 1, false, 1>(...)' -> 'k_render'."""
    n = name.replace("smoe::(anonymous namespace)::", "").split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n.split("<")[0].strip()
# Issue model: a wave64 FP32 VALU instruction occupies its SIMD for 2 cycles (32 lanes per
# cycle, the 157.3 TFLOP/s vector peak), a binary32 transcendental (v_exp_f32, v_rcp_f32, ...)
# for 8 cycles (quarter rate).
N_SIMD = 256 * 4
CLOCK_HZ = 2.4e9


def _rocpd_last(db_path, base, n):
    """Average duration (ns) of the last n dispatches of the kernel whose base name is
    `base`, in dispatch order, or None."""
    import sqlite3

    con = sqlite3.connect(db_path)
    try:
        rows = con.execute("select name, start, duration from kernels order by start").fetchall()
    except sqlite3.Error:
        return None
    finally:
        con.close()
    d = [dur for name, _, dur in rows if _kernel_base(name) == base][-n:]
    return sum(d) / len(d) if d else None


def summarize_profile(prof_dir, cmd, last=0):
    """Writes profiles/ summaries from rocprofv3 SQLite outputs under prof_dir: trace/
    (--kernel-trace --stats) and, if present, one pmc_*/ directory per --pmc run
    (FETCH_SIZE and WRITE_SIZE runs need the calibration kernel, --copy-calibration)."""
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    dbs = glob.glob(os.path.join(prof_dir, "trace", "**", "*_results.db"), recursive=True)
    durations = {}
    if dbs:
        lines = ["# rocprofv3 kernel trace: fit step and standalone binning + render, 2048x2048 "
                 "RGB, K=65536 linear experts", "",
                 f"Command: `{cmd}`", "",
                 "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
        for name, calls, tot, avg, pct in _rocpd_kernels(dbs[0]):
            short = name.replace("smoe::(anonymous namespace)::", "").split("(")[0]
            base = _kernel_base(name)
            if base in STEP_KERNELS:
                # several instantiations: the one with the most time
                if base not in durations or tot > durations[base][1]:
                    durations[base] = (avg * 1e-9, tot)
            if len(short) > 60:
                short = short[:57] + "..."
            lines.append(f"| `{short}` | {calls} | {avg / 1e3:.2f} | {tot / 1e3:.1f} | {pct:.1f} |")
        if last:
            lines += ["", f"Average of the last {last} dispatches of each step kernel (the timed "
                      "steps):", "", "| kernel | avg us |", "|---|---|"]
            for k in STEP_KERNELS:
                a = _rocpd_last(dbs[0], k, last)
                if a is not None:
                    lines.append(f"| `{k}` | {a / 1e3:.2f} |")
                    durations[k] = (a * 1e-9, float("inf"))
        gaps = _rocpd_gaps(dbs[0], list(STEP_KERNELS))
        if gaps:
            lines += ["", "Idle time between consecutive step kernels (end of one dispatch to the "
                      "start of the next):", "", "| boundary | count | median us | mean us |",
                      "|---|---|---|---|"]
            for key, v in sorted(gaps.items()):
                v = sorted(v)
                lines.append(f"| {key} | {len(v)} | {v[len(v) // 2] / 1e3:.2f} | "
                             f"{sum(v) / len(v) / 1e3:.2f} |")
        with open(os.path.join(ROOT, "profiles", "kernels_fit2048.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    ctr = {}
    for d in sorted(glob.glob(os.path.join(prof_dir, "pmc_*"))):
        for db in glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True):
            ctr.update(_rocpd_counters(db))
    if not ctr:
        return

    def per_kernel(key, counter):
        v = [x for (n, c), vals in ctr.items()
             if (_kernel_base(n) == key or key in n) and c == counter for x in vals]
        return sum(v) / len(v) if v else None

    def per_base(key, counter):
        v = [x for (n, c), vals in ctr.items() if _kernel_base(n) == key and c == counter
             for x in vals]
        return sum(v) / len(v) if v else None

    out = {"command": cmd, "calibration": None, "kernels": {}}
    f_scale = w_scale = None
    cf, cw = per_kernel("MulFunctor", "FETCH_SIZE"), per_kernel("MulFunctor", "WRITE_SIZE")
    if cf and cw:
        f_scale = CALIB_BYTES / (cf * 1024.0)
        w_scale = CALIB_BYTES / (cw * 1024.0)
        out["calibration"] = {"copy_bytes": CALIB_BYTES, "fetch_kib": cf, "write_kib": cw,
                              "fetch_scale": f_scale, "write_scale": w_scale}
    elif any(c in ("FETCH_SIZE", "WRITE_SIZE") for (_, c) in ctr):
        print("PMC byte counters lack the calibration kernel (--copy-calibration); "
              "bytes not summarised", file=sys.stderr)
    counters = sorted({c for (_, c) in ctr})
    rows = ["| kernel | avg us | fetch MB | write MB | HBM GB/s | VALU instr | VALU busy | "
            "trans busy |", "|---|---|---|---|---|---|---|---|"]
    for k, srcs in STEP_KERNELS.items():
        e = {"source_digest": source_digest(srcs), "counters": {}}
        for c in counters:
            v = per_base(k, c)
            if v is not None:
                e["counters"][c] = v
        fv, wv = e["counters"].get("FETCH_SIZE"), e["counters"].get("WRITE_SIZE")
        if f_scale and fv is not None and wv is not None:
            e["fetch_bytes"] = fv * 1024.0 * f_scale
            e["write_bytes"] = wv * 1024.0 * w_scale
        dur = durations.get(k, (None,))[0]
        if dur:
            e["avg_duration_s"] = dur
            if "fetch_bytes" in e:
                e["hbm_gbps"] = (e["fetch_bytes"] + e["write_bytes"]) / dur / 1e9
            nv = e["counters"].get("SQ_INSTS_VALU")
            nt = e["counters"].get("SQ_INSTS_VALU_TRANS_F32")
            slots = N_SIMD * CLOCK_HZ * dur
            if nv is not None:
                e["valu_busy_frac"] = nv * 2 / slots
            if nt is not None:
                e["trans_busy_frac"] = nt * 8 / slots
        if e["counters"]:
            out["kernels"][k] = e

        def f(x, scale=1.0, fmt="{:.3g}"):
            return fmt.format(x * scale) if x is not None else "-"
        rows.append(f"| `{k}` | {f(e.get('avg_duration_s'), 1e6)} | "
                    f"{f(e.get('fetch_bytes'), 1e-6)} | {f(e.get('write_bytes'), 1e-6)} | "
                    f"{f(e.get('hbm_gbps'))} | {f(e['counters'].get('SQ_INSTS_VALU'))} | "
                    f"{f(e.get('valu_busy_frac'))} | {f(e.get('trans_busy_frac'))} |")
    with open(COUNTERS_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    md = ["# rocprofv3 counters: fit step and standalone binning + render, 2048x2048 RGB, "
          "K=65536 linear experts", "",
          f"Command (trace; each pmc_* run is the same program under `--pmc <counters>`): "
          f"`{cmd}`", "",
          "Bytes: FETCH_SIZE / WRITE_SIZE per dispatch scaled by a 1 GiB elementwise kernel of "
          "known traffic.  VALU busy = SQ_INSTS_VALU x 2 cycles / (1024 SIMDs x 2.4 GHz x "
          "duration); trans busy = SQ_INSTS_VALU_TRANS_F32 x 8 cycles / the same.  Counters "
          "are summed over all XCDs and shader engines.", "",
          *rows, "", "Counters collected: " + ", ".join(counters), ""]
    with open(os.path.join(ROOT, "profiles", "counters_fit2048.md"), "w") as fh:
        fh.write("\n".join(md))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prefit", type=int, default=950,
                    help="fit steps (graph replays) before the warm-up and the timed window")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle CPU work")
    ap.add_argument("--eager", action="store_true",
                    help="no HIP graphs: every timed step is launched eagerly (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain copy of known size (for PMC byte counters)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-saturation", type=int, default=300)
    ap.add_argument("--serve-repeats", type=int, default=2,
                    help="further independent 200 req/s streams whose latencies are pooled")
    ap.add_argument("--serve-fit-steps", type=int, default=50)
    ap.add_argument("--serve-sweep-requests", type=int, default=600)
    ap.add_argument("--serve-fill-blocks", type=int, default=4096,
                    help="a batch starts beside those in flight only while they hold fewer "
                         "blocks than this")
    ap.add_argument("--serve-overlap-backlog", type=int, default=2,
                    help="queued requests needed to start a batch beside one in flight")
    ap.add_argument("--serve-one-stream", action="store_true",
                    help="also serve the Poisson stream with a one-stream batched server")
    ap.add_argument("--no-batched-fit", action="store_true")
    ap.add_argument("--bfit-steps", type=int, default=1000)
    ap.add_argument("--no-mm", action="store_true", help="skip the multi-model denoising run")
    ap.add_argument("--mm-size", type=int, default=512)
    ap.add_argument("--mm-steps", type=int, default=300)
    ap.add_argument("--no-tight", action="store_true", help="skip the square/tight box run")
    ap.add_argument("--tight-fit-steps", type=int, default=10000)
    ap.add_argument("--tight-steps", type=int, default=1000)
    ap.add_argument("--no-rbf", action="store_true", help="skip the RBF vs SMoE run")
    ap.add_argument("--rbf-steps", type=int, default=10000)
    ap.add_argument("--no-long", action="store_true", help="skip the long-list render run")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed fit, its roofline and profile (no CPU baseline and no "
                         "other section); the profiles are taken this way")
    ap.add_argument("--no-readings", action="store_true",
                    help="skip the comparison of the two truncation readings")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 64^2 and 512^2 fit workloads")
    ap.add_argument("--no-peaks", action="store_true", help="skip the issue-rate / copy probe")
    ap.add_argument("--no-autograd", action="store_true",
                    help="skip the autograd.Function run")
    ap.add_argument("--autograd-steps", type=int, default=50)
    ap.add_argument("--no-trunc-report", action="store_true",
                    help="skip the truncation-error report (oracle, untruncated vs truncated)")
    ap.add_argument("--no-early-window", action="store_true",
                    help="skip the second fit timed from the grid init")
    ap.add_argument("--summarize-profile", metavar="DIR")
    ap.add_argument("--profile-last", type=int, default=0,
                    help="also average each step kernel over its last N dispatches of the trace "
                         "(the timed steps of a run whose timed region ends the program's fit "
                         "kernels)")
    ap.add_argument("--profile-command", default="")
    args = ap.parse_args()
    if args.headline_only:
        for k in ("no_cpu_baseline", "no_serving", "no_batched_fit", "no_mm", "no_tight",
                  "no_rbf", "no_long", "no_readings", "no_small", "no_trunc_report",
                  "no_autograd", "no_peaks"):
            setattr(args, k, True)
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.profile_command, args.profile_last)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2
    run(args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
