"""Batched calls (many rasters per launch) against the oracle and against the single-raster
calls: bins bit-exact per segment after the offsets, renders bitwise equal to each raster
rendered alone, and a batched fit bitwise equal to fitting each image alone."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print("[case]", *a, flush=True)


# (width, height, scale, origin_x, origin_y, K, model index) -- a model index shared by two
# rasters renders the same resident rows at two resolutions (param_offset reuse).
RASTERS = [
    (37, 29, 1, 0, 0, 40, 0),
    (64, 48, 2, 0, 0, 120, 1),
    (16, 16, 1, 0, 0, 0, 2),        # no kernels: every block empty
    (100, 77, 3, 5, -7, 300, 3),
    (1, 1, 1, 0, 0, 3, 4),
    (120, 90, 4, 33, 10, 120, 1),   # model 1 again, another scale and window
    (55, 90, 1, 0, 0, 200, 5),
]


def build_batch(C, order, seed=0):
    """Models (one per model index) packed into one params array and the raster table."""
    models, rows = {}, []
    base = 0
    for (w, h, s, ox, oy, K, mi) in RASTERS:
        if mi not in models:
            nat_w, nat_h = max(1, w // s), max(1, h // s)
            m = wl.random_model(K, C, order, nat_w, nat_h, seed=1000 + seed * 10 + mi) if K else \
                np.zeros((0, wl.num_params(C, order)), np.float32)
            models[mi] = (base, m.astype(np.float32))
            rows.append(models[mi][1])
            base += K
    params = np.concatenate(rows) if rows else np.zeros((0, wl.num_params(C, order)), np.float32)
    rasters = [dict(width=w, height=h, scale=s, origin_x=ox, origin_y=oy, num_kernels=K,
                    param_offset=models[mi][0]) for (w, h, s, ox, oy, K, mi) in RASTERS]
    return params, rasters, models


@pytest.mark.parametrize("C,order", [(3, 1), (1, 0)])
def test_bin_batched_matches_oracle_per_segment(C, order):
    import paper_2510_05814_amd as smoe
    say("bin_batched vs oracle", C, order)
    params, rasters, models = build_batch(C, order)
    segs = smoe.Segments(rasters)
    b = smoe.bin_batched(dev(params), C, order, segs)
    over, st = b.read_status()
    assert not over
    P = st[0]
    keys = host(b.keys(P)).view(np.uint32)
    vals = host(b.vals(P)).view(np.uint32)
    ranges = host(b.ranges(segs.T))
    rects = host(b.tile_rects())
    counts = host(b.counts())
    p0 = 0
    for sg, (w, h, s, ox, oy, K, mi) in zip(segs.host, RASTERS):
        m = models[mi][1].astype(np.float64)
        o = oracle.bin(m, C, order, w, h, s, ox, oy)
        k0, t0, T = sg.kernel_offset, sg.tile_offset, oracle.blocks(w, ox) * oracle.blocks(h, oy)
        assert np.array_equal(rects[k0:k0 + K], o["tile_rects"])
        assert np.array_equal(counts[k0:k0 + K], o["counts"])
        assert np.array_equal(keys[p0:p0 + o["P"]], o["keys"] + t0)
        assert np.array_equal(vals[p0:p0 + o["P"]], o["vals"] + k0)
        assert np.array_equal(ranges[t0:t0 + T], o["ranges"] + p0)
        p0 += o["P"]
    assert p0 == P


@pytest.mark.parametrize("C,order", [(3, 1), (1, 0)])
def test_render_batched_equals_each_raster_alone(C, order, record_error):
    import torch

    import paper_2510_05814_amd as smoe
    say("render_batched vs single", C, order)
    params, rasters, models = build_batch(C, order, seed=1)
    segs = smoe.Segments(rasters)
    p = dev(params)
    b = smoe.bin_batched(p, C, order, segs)
    imgs = torch.full((segs.pixels, C), -1.0, device="cuda")
    dens = torch.full((segs.pixels,), -1.0, device="cuda")
    smoe.render_batched(p, C, order, segs, b, imgs, dens)
    worst = 0.0
    for (a, e, h, w), (_, _, s, ox, oy, K, mi) in zip(segs.pixel_slices(), RASTERS):
        grid = smoe.make_grid(w, h, s, ox, oy)
        m = dev(models[mi][1]) if K else torch.zeros((0, params.shape[1]), device="cuda")
        img1, den1, _, _ = smoe.render(m, C, order, grid)
        assert torch.equal(imgs[a:e].view(h, w, C), img1)
        assert torch.equal(dens[a:e].view(h, w), den1)
        if K:
            y_o, _ = oracle.render(models[mi][1].astype(np.float64), C, order, w, h, s, ox, oy)
            worst = max(worst, float(np.max(np.abs(host(img1) - y_o))))
    record_error(f"batched render abs C={C} order={order}", worst, 1e-5)
    assert worst <= 1e-5


def test_batched_fit_equals_individual_fits(record_error):
    """Three images of uneven sizes fitted together for 12 steps: every image's raw
    parameters, Adam moments, render and per-image loss are bitwise those of its own fit."""
    import torch

    import paper_2510_05814_amd as smoe
    say("batched fit vs individual fits")
    imgs = wl.config5_images(n=3, lo=40, hi=200)
    raws = []
    for im in imgs:
        h, w, _ = im.shape
        raw, _ = wl.grid_init(im, max(1, w // 8), max(1, h // 8), sigma=4.0, order=1)
        raws.append(raw)
    adam = smoe.AdamConfig(total_steps=12)
    steps = 12
    bst = smoe.FitState([dev(i) for i in imgs], [dev(r) for r in raws], 1, adam, max_steps=steps)
    for _ in range(steps):
        bst.step()
    seg_losses = host(bst.segment_losses())
    total = host(bst.losses())
    for i, (im, raw) in enumerate(zip(imgs, raws)):
        st = smoe.FitState(dev(im), dev(raw), 1, adam, max_steps=steps)
        for _ in range(steps):
            st.step()
        sg = bst.segments.host[i]
        k0, K = sg.kernel_offset, sg.num_kernels
        assert torch.equal(bst.raw[k0:k0 + K], st.raw), i
        assert torch.equal(bst.m[k0:k0 + K], st.m), i
        assert torch.equal(bst.v[k0:k0 + K], st.v), i
        assert torch.equal(bst.images()[i], st.image), i
        assert seg_losses[i] == host(st.segment_losses())[0], i
    assert int(host(bst.step_counter)[0]) == steps
    # the batched loss is the sum of the per-image MSEs (each a float sum over its blocks)
    err = abs(float(total[-1]) - float(seg_losses.astype(np.float64).sum())) / float(total[-1])
    record_error("batched fit loss vs sum of image losses rel", err, 1e-5)
    assert err <= 1e-5


def test_batched_fit_rejects_scaled_segments():
    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi as C
    say("batched fit validation")
    im = wl.config5_images(n=1, lo=32, hi=48)[0]
    raw, _ = wl.grid_init(im, 4, 4, order=1)
    st = smoe.FitState([dev(im)], [dev(raw)], 1, smoe.AdamConfig(total_steps=2), max_steps=2)
    st.segments.host[0].scale = 2
    with pytest.raises(C.SmoeError):
        st.step()


@pytest.mark.parametrize("mode", ["smoe", "rbf"])
def test_batched_fit_steps_against_oracle(mode, record_error):
    """The batched fit (four images of uneven sizes fitted together, the shape of the batched
    workload) against the FP64 oracle image by image: from the GPU's state before a step --
    the initial one, then after 6 more steps replayed from a HIP graph -- each image's loss, every
    gradient (per parameter group) and the Adam update of that step (the oracle's Adam from
    the GPU's own state and gradient, so that the update itself is checked)."""
    import torch

    import paper_2510_05814_amd as smoe
    say("batched fit vs oracle", mode)
    imgs = wl.config5_images(n=4, lo=40, hi=160)
    raws = wl.batched_fit_inits(imgs)
    total = 100
    adam = smoe.AdamConfig(total_steps=total)
    bst = smoe.FitState([dev(i) for i in imgs], [dev(r) for r in raws], 1, adam, max_steps=16,
                        mode=mode)
    lr_col = None
    for phase in range(2):
        if phase == 1:
            bst.replay(bst.capture(6))
        torch.cuda.synchronize()
        t = bst.steps_done()
        assert t == (0 if phase == 0 else 7)
        raw0 = host(bst.raw).astype(np.float64)
        m0, v0 = host(bst.m).astype(np.float64), host(bst.v).astype(np.float64)
        bst.step()
        torch.cuda.synchronize()
        seg = host(bst.segment_losses()).astype(np.float64)
        g_gpu = host(bst.grads).astype(np.float64)
        raw1, m1 = host(bst.raw).astype(np.float64), host(bst.m).astype(np.float64)
        lrs = oracle.step_lrs(t, total, adam.lr_mu, adam.lr_mu_final, adam.lr_chol, adam.lr_rho,
                              adam.lr_expert)
        lr_col = np.array([lrs[0]] * 2 + [lrs[1]] * 3 + [lrs[2]] + [lrs[3]] * 9)
        for i, im in enumerate(imgs):
            sg = bst.segments.host[i]
            k0, K = sg.kernel_offset, sg.num_kernels
            H, W, _ = im.shape
            rows = slice(k0, k0 + K)
            model = oracle.materialize(raw0[rows], 3, 1)
            l_o, g_o = oracle.loss_grad(model, 3, 1, W, H, target=im, rbf=(mode == "rbf"))
            el = abs(seg[i] - l_o) / l_o
            record_error(f"batched {mode} step {t} image {i} loss rel", el, 1e-5)
            assert el <= 1e-5, (i, t)
            for name, cols in {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5],
                               "a": [6, 7, 8], "wx": [9, 10, 11], "wy": [12, 13, 14]}.items():
                ref = g_o[:, cols]
                e = float(np.max(np.abs(g_gpu[rows][:, cols] - ref)) / np.max(np.abs(ref)))
                record_error(f"batched {mode} step {t} image {i} grad {name} rel", e, 1e-3)
                assert e <= 1e-3, (i, t, name)
            p, mm, vv = raw0[rows].copy(), m0[rows].copy(), v0[rows].copy()
            oracle.adam(p, g_gpu[rows], mm, vv, t + 1, lrs, 3, 1)
            ulp = np.spacing(np.abs(p).astype(np.float32)).astype(np.float64)
            d = float(np.max((np.abs(raw1[rows] - p) - ulp) / lr_col))
            record_error(f"batched {mode} step {t} image {i} Adam update beyond 1 ulp (lr)",
                         max(d, 0.0), 1e-4)
            assert d <= 1e-4, (i, t)
            em = float(np.max(np.abs(m1[rows] - mm)) / max(np.max(np.abs(mm)), 1e-30))
            assert em <= 1e-5, (i, t)
