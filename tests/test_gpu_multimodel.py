"""Multi-model fusion (block-overlapping window models, Sec. V-C): the fused image is the
per-pixel mean of the window predictions, each window's fit is the fit of that window
alone, and more hypotheses per pixel denoise better."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _noisy_clean(size=96, seed=3):
    clean, noisy = wl.config3_images(seed, H=size, W=size)
    return noisy.astype(np.float32), clean.astype(np.float32)


def test_fused_image_is_the_mean_of_window_predictions():
    import torch

    from paper_2510_05814_amd.multimodel import MultiModelDenoiser
    say("mm mean of windows")
    noisy, _ = _noisy_clean(40)
    mm = MultiModelDenoiser(noisy, 8, max_steps=5).fit(5, graphed=False)
    win = mm.window_images().cpu().numpy()
    acc = np.zeros(noisy.shape, np.float64)
    cnt = np.zeros(noisy.shape[:2], np.float64)
    p = 0
    for (y0, x0, h, w) in mm.windows:
        acc[y0:y0 + h, x0:x0 + w] += win[p:p + h * w].reshape(h, w, 3)
        cnt[y0:y0 + h, x0:x0 + w] += 1
        p += h * w
    assert np.all(cnt == mm.hypotheses)
    got = mm.image().cpu().numpy()
    assert np.max(np.abs(got - acc / cnt[..., None])) <= 1e-6
    assert torch.isfinite(mm.image()).all()


@pytest.mark.parametrize("H,W,d", [(40, 40, 8), (37, 45, 4), (20, 33, 2)])
def test_fused_image_matches_oracle(H, W, d, record_error):
    """The GPU's window models, rendered and fused by the FP64 oracle (Eq. (10)-(11)),
    against the fused image of the HIP path."""
    import oracle
    from paper_2510_05814_amd.multimodel import MultiModelDenoiser
    say("mm fused vs oracle", H, W, d)
    clean, noisy = wl.config3_images(5, H=H, W=W)
    mm = MultiModelDenoiser(noisy.astype(np.float32), d, max_steps=5).fit(5, graphed=False)
    assert mm.windows == oracle.window_rects(H, W, d)
    model = mm.state.model.cpu().numpy().astype(np.float64)
    models = [model[sg.kernel_offset:sg.kernel_offset + sg.num_kernels]
              for sg in mm.state.segments.host]
    want = oracle.fuse_windows(models, 3, 1, H, W, d)
    got = mm.image().cpu().numpy()
    e = float(np.max(np.abs(got - want)))
    record_error(f"mm fused image vs oracle {H}x{W} d={d}", e, 1e-5)
    assert e <= 1e-5


def test_fusion_is_a_fixed_order_binary32_mean():
    """smoe_fuse_windows sums the covering windows in (window row, window column) order in
    binary32 and divides by the hypothesis count (correctly rounded, also for a count that is
    not a power of two): bitwise the same sums done on the host in that order, and bitwise the
    same on every call."""
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.multimodel import window_layout
    say("mm fusion fixed order")
    rng = np.random.default_rng(11)
    for (H, W, d, C, win) in [(37, 45, 4, 3, 16), (20, 33, 2, 1, 16), (16, 16, 16, 3, 16),
                              (5, 7, 4, 1, 16), (29, 31, 4, 3, 12)]:
        m = win // d
        rects = window_layout(H, W, d, win)
        wins = [rng.uniform(-1, 1, (h, w, C)).astype(np.float32) for (_, _, h, w) in rects]
        flat = np.concatenate([x.reshape(-1, C) for x in wins])
        assert flat.shape[0] == m * m * W * H
        acc = np.zeros((H, W, C), np.float32)
        for (y0, x0, h, w), x in zip(rects, wins):
            acc[y0:y0 + h, x0:x0 + w] += x
        want = acc / np.float32(m * m)
        dev = torch.from_numpy(flat).cuda()
        a = smoe.fuse_windows(dev, C, W, H, d, win)
        b = smoe.fuse_windows(dev, C, W, H, d, win)
        assert torch.equal(a, b)
        assert np.array_equal(a.cpu().numpy(), want), (H, W, d, C, win)


def test_each_window_fit_is_its_own_fit():
    """Window fits in the batch equal fitting each window alone, bitwise."""
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.multimodel import MultiModelDenoiser, _grid_init
    say("mm windows independent")
    noisy, _ = _noisy_clean(48)
    adam = smoe.AdamConfig(total_steps=6)
    mm = MultiModelDenoiser(noisy, 16, adam=adam, max_steps=6).fit(6, graphed=False)
    st = mm.state
    for i in (0, 4, len(mm.windows) - 1):
        y0, x0, h, w = mm.windows[i]
        crop = np.ascontiguousarray(noisy[y0:y0 + h, x0:x0 + w])
        raw = _grid_init(crop, 8, 4.0, 1)
        one = smoe.FitState(torch.from_numpy(crop).cuda(), torch.from_numpy(raw).cuda(), 1,
                            adam, max_steps=6)
        for _ in range(6):
            one.step()
        sg = st.segments.host[i]
        assert torch.equal(st.raw[sg.kernel_offset:sg.kernel_offset + sg.num_kernels], one.raw)


def test_more_hypotheses_denoise_better(record_error):
    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.multimodel import MultiModelDenoiser
    say("mm psnr vs hypotheses")
    noisy, clean = _noisy_clean(96)
    import torch
    c = torch.from_numpy(clean).cuda()
    ps = {}
    for d in (16, 4):
        mm = MultiModelDenoiser(noisy, d, adam=smoe.AdamConfig(total_steps=200)).fit(200)
        ps[d] = smoe.psnr(mm.image(), c)
    print("[mm] psnr", ps, flush=True)
    assert ps[4] > ps[16] + 0.3
