"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: block rectangles, counts, P, keys, kernel order and ranges bit-exact; images within
1e-5 absolute and D within 1e-5 relative; gradients within 1e-3 (max error over a
parameter group relative to the group's largest oracle gradient); losses within 1e-5
relative.  Every measured error is recorded with its bound.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

Y_TOL = 1e-5
from tests._tol import D_RTOL, d_rel_error
G_TOL = 1e-3


@pytest.fixture(scope="module")
def smoe():
    import torch  # noqa: F401

    import paper_2510_05814_amd as smoe
    return smoe


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def groups(C, order):
    g = {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5], "a": list(range(6, 6 + C))}
    if order == 1:
        g["wx"] = list(range(6 + C, 6 + 2 * C))
        g["wy"] = list(range(6 + 2 * C, 6 + 3 * C))
    return g


def say(*a):
    print("[case]", *a, flush=True)


def gpu_bins(smoe, model_np, C, order, grid):
    m = dev(model_np)
    b = smoe.bin(m, C, order, grid)
    over, st = b.read_status()
    assert not over
    P = st[0]
    T = smoe.tiles(grid.width, grid.height, grid.origin_x, grid.origin_y)
    return m, b, dict(tile_rects=host(b.tile_rects()), native_rects=host(b.native_rects()),
                      counts=host(b.counts()), P=P,
                      keys=host(b.keys(P)).view(np.uint32), vals=host(b.vals(P)).view(np.uint32),
                      ranges=host(b.ranges(T)), longest=st[2])


def assert_bins_equal(g, o):
    assert g["P"] == o["P"]
    assert np.array_equal(g["tile_rects"], o["tile_rects"])
    assert np.array_equal(g["native_rects"], o["native_rects"])
    assert np.array_equal(g["counts"], o["counts"])
    assert np.array_equal(g["keys"], o["keys"])
    assert np.array_equal(g["vals"], o["vals"])
    assert np.array_equal(g["ranges"], o["ranges"])


RANDOM_CASES = [
    # (W, H, K, C, order, seed, sig_lo, sig_hi)
    (37, 29, 40, 1, 0, 101, 1.0, 9.0),
    (64, 48, 120, 3, 1, 102, 0.6, 12.0),
    (100, 77, 300, 3, 0, 103, 0.8, 6.0),
    (55, 90, 200, 1, 1, 104, 0.5, 20.0),
    (1, 1, 3, 3, 1, 105, 0.5, 3.0),
    (17, 16, 1, 3, 1, 106, 2.0, 4.0),
]


@pytest.mark.parametrize("case", RANDOM_CASES, ids=[f"{c[0]}x{c[1]}K{c[2]}C{c[3]}o{c[4]}" for c in RANDOM_CASES])
def test_bin_and_render_random_models(smoe, case, record_error):
    W, H, K, C, order, seed, lo, hi = case
    say("random", case)
    m_np = wl.random_model(K, C, order, W, H, seed, sig_lo=lo, sig_hi=hi)
    grid = smoe.make_grid(W, H)
    m, b, gb = gpu_bins(smoe, m_np, C, order, grid)
    ob = oracle.bin(m_np, C, order, W, H)
    assert_bins_equal(gb, ob)
    img, D, _, _ = smoe.render(m, C, order, grid, bins=b)
    y_o, D_o = oracle.render(m_np, C, order, W, H)
    ey = np.max(np.abs(host(img) - y_o))
    eD = d_rel_error(host(D), D_o)
    record_error("image abs", ey, Y_TOL)
    record_error("denominator rel (exponent-scaled)", eD, D_RTOL)
    assert ey <= Y_TOL and eD <= D_RTOL
    assert np.array_equal(host(D) > 0, D_o > 0)


SUBPIXEL = [(2, 0, 0), (3, 5, 7), (4, 13, 2), (3, 0, 0)]


@pytest.mark.parametrize("s,ox,oy", SUBPIXEL)
def test_subpixel_grids(smoe, s, ox, oy, record_error):
    say("subpixel", s, ox, oy)
    W, H = 40, 31
    m_np = wl.random_model(60, 3, 1, W, H, seed=200 + s, sig_lo=0.8, sig_hi=7.0)
    OW, OH = s * W - ox, s * H - oy
    grid = smoe.make_grid(OW, OH, s, ox, oy)
    m, b, gb = gpu_bins(smoe, m_np, 3, 1, grid)
    assert_bins_equal(gb, oracle.bin(m_np, 3, 1, OW, OH, s, ox, oy))
    img, D, _, _ = smoe.render(m, 3, 1, grid, bins=b)
    y_o, D_o = oracle.render(m_np, 3, 1, OW, OH, s, ox, oy)
    ey = np.max(np.abs(host(img) - y_o))
    record_error("image abs", ey, Y_TOL)
    assert ey <= Y_TOL


def test_long_lists_chunked_and_merged(smoe, record_error):
    """Block lists longer than one LDS chunk (256) and than one sort run (2048)."""
    W, H = 48, 40
    K = 2600
    rng = np.random.default_rng(7)
    m_np = wl.random_model(K, 3, 1, W, H, seed=300, sig_lo=6.0, sig_hi=30.0, margin=-4.0)
    m_np[:, 5] = rng.normal(0, 0.3, K)
    say("long lists", K)
    grid = smoe.make_grid(W, H)
    m, b, gb = gpu_bins(smoe, m_np, 3, 1, grid)
    ob = oracle.bin(m_np, 3, 1, W, H)
    assert gb["longest"] > 2048
    assert_bins_equal(gb, ob)
    img, D, _, _ = smoe.render(m, 3, 1, grid, bins=b)
    y_o, _ = oracle.render(m_np, 3, 1, W, H)
    ey = np.max(np.abs(host(img) - y_o))
    record_error("image abs", ey, Y_TOL)
    assert ey <= Y_TOL


def test_empty_model_and_uncovered_pixels(smoe):
    say("empty")
    import torch
    grid = smoe.make_grid(33, 20)
    m = torch.zeros((0, 15), dtype=torch.float32, device="cuda")
    b = smoe.bin(m, 3, 1, grid)
    img, D, _, _ = smoe.render(m, 3, 1, grid, bins=b)
    assert torch.all(img == 0) and torch.all(D == 0)
    # all kernels far outside the raster
    m_np = wl.random_model(10, 3, 1, 33, 20, seed=5)
    m_np[:, 0] += 500.0
    m2 = dev(m_np)
    b2 = smoe.bin(m2, 3, 1, grid)
    _, st = b2.read_status()
    assert st[0] == 0
    img2, D2, _, _ = smoe.render(m2, 3, 1, grid, bins=b2)
    assert torch.all(img2 == 0)


def test_workloads_at_full_size(smoe, record_error):
    """The 64^2 and 512^2 fit workloads and the 2048^2 K=65536 workload at init: bins
    bit-exact; image compared everywhere (64^2, 512^2) or on 3000 sampled pixels (2048^2)."""
    for n in (1, 2, 3):
        w = wl.workload(n)
        H, W, C = w.target.shape
        say("workload", n, w.name)
        model_np = w.raw0.copy()
        model_np[:, 2] = np.exp(model_np[:, 2].astype(np.float64)).astype(np.float32)
        model_np[:, 4] = np.exp(model_np[:, 4].astype(np.float64)).astype(np.float32)
        grid = smoe.make_grid(W, H)
        m, b, gb = gpu_bins(smoe, model_np, C, w.order, grid)
        ob = oracle.bin(model_np, C, w.order, W, H)
        assert_bins_equal(gb, ob)
        img, D, loss, _ = smoe.render(m, C, w.order, grid, bins=b, target=dev(w.target))
        if n < 3:
            y_o, D_o = oracle.render(model_np, C, w.order, W, H)
            gi = host(img)
            ey = np.max(np.abs(gi - y_o))
            l_o = np.mean((y_o - w.target) ** 2)
            el = abs(loss.item() - l_o) / l_o
            record_error(f"workload {n} loss rel", el, 1e-5)
            assert el <= 1e-5
        else:
            rng = np.random.default_rng(11)
            pix = np.stack([rng.integers(0, W, 3000), rng.integers(0, H, 3000)], 1)
            pix = np.concatenate([pix, [[0, 0], [W - 1, H - 1], [W - 1, 0], [0, H - 1]]])
            y_o, D_o = oracle.render(model_np, C, w.order, W, H, pixels=pix)
            gi = host(img)[pix[:, 1], pix[:, 0]]
            ey = np.max(np.abs(gi - y_o))
        record_error(f"workload {n} image abs", ey, Y_TOL)
        assert ey <= Y_TOL


def test_gates_sum_to_one_bitwise(smoe):
    """All-ones constant experts: N and D get the same addends in the same order, so y is
    exactly 1 wherever D > 0."""
    say("gates sum")
    W, H = 70, 50
    m_np = wl.random_model(150, 3, 1, W, H, seed=41)
    m_np[:, 6:9] = 1.0
    m_np[:, 9:] = 0.0
    m = dev(m_np)
    img, D, _, _ = smoe.render(m, 3, 1, smoe.make_grid(W, H))
    gi, gD = host(img), host(D)
    assert (gD > 0).any()
    assert np.all(gi[gD > 0] == 1.0) and np.all(gi[gD == 0] == 0.0)


def test_translation_equivariance_bitwise(smoe):
    say("translation")
    W, H = 64, 48
    m_np = wl.random_model(40, 3, 1, W, H, seed=43, margin=-8.0)
    m_np[:, :2] = np.round(m_np[:, :2] * 256) / 256
    # any integer shift with the ellipse test in the render; whole blocks when the block
    # lists alone decide the render
    for trunc, (tx, ty) in (("render", (5, 3)), ("gradient", (16, 32))):
        img0, _, _, _ = smoe.render(dev(m_np), 3, 1, smoe.make_grid(W, H, trunc=trunc))
        m2 = m_np.copy()
        m2[:, 0] += tx
        m2[:, 1] += ty
        img1, _, _, _ = smoe.render(dev(m2), 3, 1, smoe.make_grid(W + tx, H + ty, trunc=trunc))
        assert np.array_equal(host(img1)[ty:, tx:], host(img0)), trunc


def test_render_and_backward_deterministic(smoe):
    """Two runs give bitwise identical images and gradients (no atomics in any sum)."""
    say("determinism")
    tgt, raw = wl.fd_crop_case(seed=12)
    model_np = oracle.materialize(raw, 3, 1).astype(np.float32)
    m, t = dev(model_np), dev(tgt)
    grid = smoe.make_grid(32, 32)
    outs = []
    for _ in range(2):
        img, D, loss, b = smoe.render(m, 3, 1, grid, target=t)
        g = smoe.render_backward(m, 3, 1, grid, b, img, D, target=t)
        outs.append((host(img), host(g), loss.item()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def check_grads(g_gpu, g_ref, C, order, record_error, label):
    for name, cols in groups(C, order).items():
        ref = g_ref[:, cols]
        scale = np.max(np.abs(ref))
        if scale == 0:
            assert np.max(np.abs(g_gpu[:, cols])) == 0
            continue
        err = np.max(np.abs(g_gpu[:, cols] - ref)) / scale
        record_error(f"{label} grad {name} rel", err, G_TOL)
        assert err <= G_TOL, (name, err)


GRAD_CASES = ["crop", "workload1", "workload2", "random3", "random1"]


@pytest.mark.parametrize("case", GRAD_CASES)
def test_backward_mse_against_oracle(smoe, case, record_error):
    say("grad", case)
    if case == "crop":
        tgt, raw = wl.fd_crop_case()
        C, order = 3, 1
        model_np = oracle.materialize(raw, 3, 1).astype(np.float32)
    elif case.startswith("workload"):
        w = wl.workload(int(case[-1]))
        tgt, C, order = w.target, w.target.shape[2], w.order
        rng = np.random.default_rng(3)
        raw = w.raw0.astype(np.float64)
        raw[:, :2] += rng.uniform(-2, 2, (w.K, 2))
        raw[:, 2] += rng.uniform(-0.3, 0.3, w.K)
        raw[:, 3] = rng.uniform(-1, 1, w.K)
        model_np = oracle.materialize(raw, C, order).astype(np.float32)
    else:
        C = int(case[-1])
        order = 1
        W, H = 53, 45
        model_np = wl.random_model(90, C, order, W, H, seed=77 + C)
        tgt = np.random.default_rng(C).uniform(0, 1, (H, W, C)).astype(np.float32)
    H, W, _ = tgt.shape
    grid = smoe.make_grid(W, H)
    m, t = dev(model_np), dev(tgt)
    img, D, loss, b = smoe.render(m, C, order, grid, target=t)
    g = host(smoe.render_backward(m, C, order, grid, b, img, D, target=t))
    l_o, g_o = oracle.loss_grad(model_np, C, order, W, H, target=tgt)
    el = abs(loss.item() - l_o) / l_o
    record_error(f"{case} loss rel", el, 1e-5)
    assert el <= 1e-5
    check_grads(g, g_o, C, order, record_error, case)


def test_backward_upstream_gradient_mode(smoe, record_error):
    say("grad_y mode")
    W, H = 45, 38
    model_np = wl.random_model(70, 3, 1, W, H, seed=88)
    gy = np.random.default_rng(9).normal(0, 1e-3, (H, W, 3)).astype(np.float32)
    grid = smoe.make_grid(W, H)
    m = dev(model_np)
    img, D, _, b = smoe.render(m, 3, 1, grid)
    g = host(smoe.render_backward(m, 3, 1, grid, b, img, D, grad_image=dev(gy)))
    _, g_o = oracle.loss_grad(model_np, 3, 1, W, H, grad_y=gy)
    check_grads(g, g_o, 3, 1, record_error, "grad_y")


def test_backward_full_size_sampled_kernels(smoe, record_error):
    """2048^2, K = 65536 (perturbed from the grid init): gradients of 24 sampled kernels
    against the oracle, which evaluates exactly the pixels of those kernels' blocks."""
    w = wl.workload(3)
    H, W, C = w.target.shape
    rng = np.random.default_rng(21)
    raw = w.raw0.astype(np.float64)
    raw[:, :2] += rng.uniform(-2, 2, (w.K, 2))
    raw[:, 3] = rng.uniform(-1, 1, w.K)
    raw[:, 9:] = rng.uniform(-0.01, 0.01, (w.K, 6))
    model_np = oracle.materialize(raw, C, 1).astype(np.float32)
    say("full-size grads")
    grid = smoe.make_grid(W, H)
    m, t = dev(model_np), dev(w.target)
    img, D, loss, b = smoe.render(m, C, 1, grid, target=t)
    g = host(smoe.render_backward(m, C, 1, grid, b, img, D, target=t))
    sel = np.concatenate([[0, w.K - 1, 255, w.K - 256], rng.choice(w.K, 20, replace=False)])
    _, g_o = oracle.loss_grad(model_np, C, 1, W, H, target=w.target, kernels=sel)
    check_grads(g[sel], g_o, C, 1, record_error, "2048 sampled")


def test_fit_step_full_size_after_graphed_steps(smoe, record_error):
    """The fused fit step in the configuration the benchmark times (2048^2 RGB, K = 65536,
    the fit state's own bucket width, steps replayed from HIP graphs): after 40 steps, one more
    step's render (of the model it starts from) at every pixel and its gradient of 24
    sampled kernels against the oracle on that model."""
    import torch
    say("full-size fit step")
    w = wl.workload(3)
    H, W, C = w.target.shape
    target = dev(w.target)
    raw0 = dev(w.raw0)
    b0 = smoe.bin(smoe.materialize(raw0, C, 1), C, 1, smoe.make_grid(W, H))
    P0 = b0.read_status()[1][0]
    st = smoe.FitState(target, raw0, 1, smoe.AdamConfig(total_steps=10000), max_steps=64)
    assert st.bins.capacity == smoe.tiles(W, H) * 64  # one-chunk buckets: the short kernel
    assert P0 > 0
    st.run_graphed(40)
    model_np = host(st.model).copy()
    st.step()
    torch.cuda.synchronize()
    assert not st.bins.read_status()[0]
    rng = np.random.default_rng(31)
    # the whole 2048^2 image (the oracle takes ~20 s on 16 threads)
    y_o, _ = oracle.render(model_np, C, 1, W, H)
    ey = float(np.max(np.abs(host(st.image) - y_o)))
    record_error("full-size fit step image abs (every pixel)", ey, Y_TOL)
    assert ey <= Y_TOL
    sel = np.concatenate([[0, w.K - 1], rng.choice(w.K, 22, replace=False)])
    _, g_o = oracle.loss_grad(model_np, C, 1, W, H, target=w.target, kernels=sel)
    check_grads(host(st.grads)[sel], g_o, C, 1, record_error, "full-size fit step sampled")


def test_fit_step_one_step_against_oracle_adam(smoe, record_error):
    """One smoe_fit_step from the same raw state: the loss, the gradient and the Adam update
    (within the propagated gradient tolerance) against the oracle's FP64 pieces."""
    import torch
    say("fit one step")
    w = wl.workload(2)
    H, W, C = w.target.shape
    adam = smoe.AdamConfig(total_steps=2000)
    st = smoe.FitState(dev(w.target), dev(w.raw0), 1, adam, max_steps=4)
    loss = torch.zeros(1, device="cuda")
    st.step(loss)
    raw_gpu, g_gpu = host(st.raw), host(st.grads)
    raw0 = w.raw0.astype(np.float64)
    model0 = oracle.materialize(raw0, C, 1)
    l_o, g_o = oracle.loss_grad(model0, C, 1, W, H, target=w.target)
    el = abs(loss.item() - l_o) / l_o
    record_error("fit step loss rel", el, 1e-5)
    assert el <= 1e-5 and st.steps_done() == 1
    check_grads(g_gpu, g_o, C, 1, record_error, "fit step")
    p, mm, vv = raw0.copy(), np.zeros_like(raw0), np.zeros_like(raw0)
    lrs = oracle.step_lrs(0, 2000, adam.lr_mu, adam.lr_mu_final, adam.lr_chol, adam.lr_rho,
                          adam.lr_expert)
    oracle.adam(p, g_o, mm, vv, 1, lrs, C, 1)
    # First Adam step moves each parameter by lr * g / (|g| + eps): compare where the
    # gradient is well above the gradient tolerance of its group; elsewhere the step is
    # bounded by lr.
    # The new value is stored in FP32, so one ulp of it is added to the bound (an ulp of
    # a centre near 500 px is 6e-5 px, several thousandths of the 0.01 px step).
    lr_col = np.array([lrs[0]] * 2 + [lrs[1]] * 3 + [lrs[2]] + [lrs[3]] * 9)
    ulp = np.spacing(np.abs(p).astype(np.float32)).astype(np.float64)
    step_gpu = raw_gpu - w.raw0.astype(np.float64)
    for name, cols in groups(C, 1).items():
        scale = np.max(np.abs(g_o[:, cols]))
        sig = np.abs(g_o[:, cols]) > 1e-2 * scale
        d = (np.abs(raw_gpu[:, cols] - p[:, cols]) - ulp[:, cols]) / lr_col[cols]
        e = max(0.0, np.max(d[sig])) if sig.any() else 0.0
        record_error(f"adam step {name} beyond 1 ulp (units of lr)", e, 1e-3)
        assert e <= 1e-3
        assert np.all(np.abs(step_gpu[:, cols]) <= lr_col[cols] * 1.0001 + ulp[:, cols])
    mod = host(st.model)
    np.testing.assert_allclose(mod[:, 2], np.exp(raw_gpu[:, 2]), rtol=3e-7)
    np.testing.assert_allclose(mod[:, 4], np.exp(raw_gpu[:, 4]), rtol=3e-7)


def test_fit_workload1_100_steps_loss_curve(smoe, record_error):
    """100 Adam steps on the 64^2 grey workload: loss curve within 1e-3 relative of the FP64
    oracle's fit and final PSNR within 0.01 dB.  (FP32 and FP64 trajectories drift apart
    slowly; this bounds the drift over the workload's full length.)"""
    say("fit 100")
    w = wl.workload(1)
    adam = smoe.AdamConfig.constant(1e-2, total_steps=100)
    st = smoe.FitState(dev(w.target), dev(w.raw0), 0, adam, max_steps=100)
    st.run(100)
    hist = host(st.losses())
    h_o, raw_o = oracle.fit(w.raw0, 1, 0, w.target, steps=100, lr_mu=1e-2, lr_chol=1e-2,
                            lr_rho=1e-2, lr_expert=1e-2)
    e = np.max(np.abs(hist - h_o) / h_o)
    record_error("loss curve rel", e, 1e-3)
    assert e <= 1e-3
    final_gpu = 10 * math.log10(1.0 / float(hist[-1]))
    final_o = 10 * math.log10(1.0 / h_o[-1])
    record_error("PSNR at last step dB", abs(final_gpu - final_o), 0.01)
    assert abs(final_gpu - final_o) <= 0.01
    assert hist[-1] < 0.7 * hist[0]


def test_capacity_overflow_is_reported_and_harmless(smoe):
    """Too small a pair capacity: the status gives the exact P needed, every block list is
    empty (zeros render) and a fit step changes nothing, step counter included."""
    import torch
    say("overflow")
    w = wl.workload(1)
    H, W, C = w.target.shape
    model_np = w.raw0.copy()
    model_np[:, 2] = 4.0
    model_np[:, 4] = 4.0
    m = dev(model_np)
    grid = smoe.make_grid(W, H)
    b = smoe.Bins(64, 1, 0, smoe.tiles(W, H), 10, "cuda")
    smoe.bin(m, 1, 0, grid, bins=b, grow=False)
    over, st = b.read_status()
    assert over and st[0] == oracle.bin(model_np, 1, 0, W, H)["P"]
    img, D, _, _ = smoe.render(m, 1, 0, grid, bins=b)
    assert torch.all(img == 0)
    fs = smoe.FitState(dev(w.target), dev(w.raw0), 0, smoe.AdamConfig.constant(1e-2), capacity=10)
    raw_before = fs.raw.clone()
    fs.step()
    assert fs.steps_done() == 0 and torch.equal(fs.raw, raw_before)
    assert fs.grow_if_needed()
    fs.step()
    assert fs.steps_done() == 1 and not torch.equal(fs.raw, raw_before)


def test_fused_fit_step_equals_standalone_calls(smoe):
    """The fit step's fused kernels (bucket sort inside the render, next-step binning inside
    Adam) give bitwise the image and gradient of smoe_bin + smoe_render +
    smoe_render_backward, on the first step (prologue binning) and on later steps (binning
    left by the previous step's Adam)."""
    import torch
    say("fused vs standalone")
    w = wl.workload(2)
    H, W, C = w.target.shape
    t = dev(w.target)
    st = smoe.FitState(t, dev(w.raw0), 1, smoe.AdamConfig(total_steps=2000), max_steps=8)
    grid = smoe.make_grid(W, H)
    for k in range(3):
        model = st.model.clone()
        img, D, _, b = smoe.render(model, C, 1, grid)
        g = smoe.render_backward(model, C, 1, grid, b, img, D, target=t)
        st.step()
        torch.cuda.synchronize()
        assert torch.equal(st.image, img), k
        assert torch.equal(st.denom, D), k
        assert torch.equal(st.grads, g), k

FUSED_SHAPES = [(1, 0, "smoe", 301), (3, 0, "smoe", 302), (1, 1, "smoe", 303),
                (3, 1, "rbf", 304), (1, 0, "rbf", 305)]


@pytest.mark.parametrize("C_,order,mode,seed", FUSED_SHAPES)
def test_fused_fit_step_equals_standalone_calls_shapes(smoe, C_, order, mode, seed):
    """The same bitwise equality for the other expert shapes and the RBF mode: the gather's
    per-kernel finishing (the centre's expert-slope terms) is shared by the fit step's Adam
    and the standalone gather, which take the slopes from the raw row and the render record."""
    import torch
    say(f"fused vs standalone C={C_} order={order} {mode}")
    W, H, K = 96, 80, 150
    m_np = wl.random_model(K, C_, order, W, H, seed, sig_lo=1.5, sig_hi=8.0)
    raw = m_np.astype(np.float64).copy()
    raw[:, 2], raw[:, 4] = np.log(m_np[:, 2]), np.log(m_np[:, 4])
    t = dev(np.random.default_rng(seed).uniform(0, 1, (H, W, C_)).astype(np.float32))
    st = smoe.FitState(t, dev(raw), order, smoe.AdamConfig(total_steps=100), max_steps=8,
                       mode=mode)
    grid = smoe.make_grid(W, H, mode=mode)
    for k in range(3):
        model = st.model.clone()
        img, D, _, b = smoe.render(model, C_, order, grid)
        g = smoe.render_backward(model, C_, order, grid, b, img, D, target=t)
        st.step()
        torch.cuda.synchronize()
        assert torch.equal(st.image, img), k
        assert torch.equal(st.denom, D), k
        assert torch.equal(st.grads, g), k

