"""The RBF mode (Eq. 1: the un-normalised weighted sum of kernels) on the GPU, against the
oracle's RBF mode.  Bars: block lists are those of the gated mode (same boxes, bit for bit);
images within 1e-5 of the oracle relative to the image's peak magnitude (Eq. 1 is not bounded
by the experts' range as the gated mixture is); gradients within 1e-3 relative to the largest
oracle gradient of their group; losses within 1e-5 relative; batched renders bitwise equal to
single renders."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests._tol import d_rel_error

pytestmark = pytest.mark.gpu

Y_TOL = 1e-5
G_TOL = 1e-3
GROUPS1 = {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5]}


def say(*a):
    print("[case]", *a, flush=True)


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


def rbf_model(K, C, order, W, H, seed):
    """A random model whose kernel weights pi are around e^-1, so that the sum of Eq. (1)
    stays O(1) where a few kernels overlap."""
    m = wl.random_model(K, C, order, W, H, seed, sig_lo=0.7, sig_hi=8.0, rho_std=0.3)
    m[:, 5] -= 1.0
    return m


def groups(C, order):
    g = dict(GROUPS1, a=list(range(6, 6 + C)))
    if order == 1:
        g["wx"] = list(range(6 + C, 6 + 2 * C))
        g["wy"] = list(range(6 + 2 * C, 6 + 3 * C))
    return g


def check_grads(g, ref, C, order, record_error, label):
    for name, cols in groups(C, order).items():
        scale = float(np.max(np.abs(ref[:, cols])))
        if scale == 0:
            assert np.max(np.abs(g[:, cols])) == 0
            continue
        e = float(np.max(np.abs(g[:, cols] - ref[:, cols]))) / scale
        record_error(f"{label} grad {name} rel", e, G_TOL)
        assert e <= G_TOL, (name, e)


CASES = [
    # (W, H, K, C, order, scale, origin_x, origin_y, seed)
    (53, 41, 120, 3, 1, 1, 0, 0, 601),
    (37, 29, 40, 1, 0, 1, 0, 0, 602),
    (40, 31, 60, 3, 0, 3, 5, 7, 603),
    (64, 48, 200, 1, 1, 2, 0, 0, 604),
    (1, 1, 3, 3, 1, 1, 0, 0, 605),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}K{c[2]}C{c[3]}o{c[4]}s{c[5]}" for c in CASES])
def test_rbf_render_against_oracle(smoe, case, record_error):
    W, H, K, C, order, s, ox, oy, seed = case
    say("rbf render", case)
    m_np = rbf_model(K, C, order, W, H, seed)
    OW, OH = s * W - ox, s * H - oy
    m = dev(m_np)
    grid = smoe.make_grid(OW, OH, s, ox, oy, mode="rbf")
    img, D, _, b = smoe.render(m, C, order, grid)
    y_o, D_o = oracle.render(m_np, C, order, OW, OH, s, ox, oy, rbf=True)
    peak = max(1.0, float(np.max(np.abs(y_o))))
    ey = float(np.max(np.abs(host(img) - y_o))) / peak
    record_error("rbf image abs / peak", ey, Y_TOL)
    assert ey <= Y_TOL
    eD = d_rel_error(host(D), D_o)
    assert eD <= 1e-5
    # the same block lists as the gated mode
    _, st = b.read_status()
    ob = oracle.bin(m_np, C, order, OW, OH, s, ox, oy)
    assert st[0] == ob["P"]
    assert np.array_equal(host(b.vals(st[0])).view(np.uint32), ob["vals"])


@pytest.mark.parametrize("C,order", [(3, 1), (1, 0)])
def test_rbf_backward_against_oracle(smoe, C, order, record_error):
    say("rbf backward", C, order)
    W, H = 61, 47
    m_np = rbf_model(150, C, order, W, H, 610 + C)
    t_np = np.random.default_rng(C).uniform(0, 1, (H, W, C)).astype(np.float32)
    m, t = dev(m_np), dev(t_np)
    grid = smoe.make_grid(W, H, mode="rbf")
    img, D, loss, b = smoe.render(m, C, order, grid, target=t)
    g = host(smoe.render_backward(m, C, order, grid, b, img, D, target=t))
    l_o, g_o = oracle.loss_grad(m_np, C, order, W, H, target=t_np, rbf=True)
    el = abs(loss.item() - l_o) / l_o
    record_error("rbf loss rel", el, 1e-5)
    assert el <= 1e-5
    check_grads(g, g_o, C, order, record_error, "rbf")
    # upstream-gradient mode
    gy_np = np.random.default_rng(7).normal(0, 1, (H, W, C)).astype(np.float32)
    g2 = host(smoe.render_backward(m, C, order, grid, b, img, D, grad_image=dev(gy_np)))
    _, g2_o = oracle.loss_grad(m_np, C, order, W, H, grad_y=gy_np, rbf=True)
    check_grads(g2, g2_o, C, order, record_error, "rbf grad_y")


def test_rbf_fit_step_against_oracle(smoe, record_error):
    """One fused fit step in the RBF mode: its loss and gradient against the oracle's."""
    import torch
    say("rbf fit step")
    W, H = 72, 56
    img_np = wl.step_edge_image(seed=5, H=H, W=W, C=3)
    raw, _ = wl.grid_init(img_np, 9, 7, 4.0, order=1)
    raw = raw.astype(np.float64)
    raw[:, 5] = -0.5
    st = smoe.FitState(dev(img_np), dev(raw), 1, smoe.AdamConfig(total_steps=10), max_steps=4,
                       mode="rbf")
    loss = torch.zeros(1, device="cuda")
    st.step(loss)
    model0 = oracle.materialize(raw, 3, 1)
    l_o, g_o = oracle.loss_grad(model0, 3, 1, W, H, target=img_np, rbf=True)
    el = abs(loss.item() - l_o) / l_o
    record_error("rbf fit step loss rel", el, 1e-5)
    assert el <= 1e-5
    check_grads(host(st.grads), g_o, 3, 1, record_error, "rbf fit step")


def test_rbf_batched_equals_single(smoe):
    import torch
    say("rbf batched")
    models = [rbf_model(K, 3, 1, 36, 30, 620 + K) for K in (40, 90)]
    params = dev(np.concatenate(models))
    specs = [(0, 1, 0, 0), (1, 2, 3, 1), (0, 3, 0, 5)]
    rasters = [dict(width=36 * s - ox, height=30 * s - oy, scale=s, origin_x=ox, origin_y=oy,
                    num_kernels=models[i].shape[0], param_offset=0 if i == 0 else 40)
               for i, s, ox, oy in specs]
    segs = smoe.Segments(rasters)
    bins = smoe.bin_batched(params, 3, 1, segs, mode="rbf")
    out = torch.empty((segs.pixels, 3), dtype=torch.float32, device="cuda")
    smoe.render_batched(params, 3, 1, segs, bins, out, mode="rbf")
    for (a, e, h, w), (i, s, ox, oy) in zip(segs.pixel_slices(), specs):
        alone, _, _, _ = smoe.render(dev(models[i]), 3, 1,
                                     smoe.make_grid(w, h, s, ox, oy, mode="rbf"))
        assert torch.equal(out[a:e].view(h, w, 3), alone), (i, s)


def test_rbf_batched_fit_equals_individual_fits(smoe):
    """Two images fitted together in the RBF mode, bit for bit the images fitted alone."""
    import torch
    say("rbf batched fit")
    imgs = [wl.step_edge_image(seed=s, H=h, W=w, C=3) for s, h, w in ((41, 48, 64), (42, 40, 40))]
    raws = []
    for im in imgs:
        raw, _ = wl.grid_init(im, 6, 5, 4.0, order=1)
        raw[:, 5] = -0.5
        raws.append(raw)
    adam = smoe.AdamConfig(total_steps=20)
    tg = [torch.from_numpy(i) for i in imgs]
    rw = [torch.from_numpy(r) for r in raws]
    both = smoe.FitState(tg, rw, 1, adam, max_steps=21, mode="rbf")
    both.run(20)
    alone = []
    for t, r in zip(tg, rw):
        st = smoe.FitState(t.cuda(), r.cuda(), 1, adam, max_steps=21, mode="rbf")
        st.run(20)
        alone.append(st)
    torch.cuda.synchronize()
    for (a, e, h, w), st in zip(both.segments.pixel_slices(), alone):
        assert torch.equal(both.image[a:e].view(h, w, 3), st.image)


def test_rbf_serving_equals_alone(smoe):
    """A model bank in the RBF mode: batched and plain servers give each request the image of
    rendering it alone."""
    import torch

    from paper_2510_05814_amd.serve import ModelBank, PlainServer, RenderRequest, Server
    say("rbf serving")
    models = [rbf_model(K, 3, 1, 48, 40, 630 + K).astype(np.float32) for K in (70, 130)]
    bank = ModelBank(models, 3, 1, mode="rbf")
    reqs = [RenderRequest(i % 2, 1 + i % 3, 40 + 7 * i, 33 + 5 * i, i, 2 * i, arrival=0.0)
            for i in range(6)]
    res, _ = Server(bank, streams=2).serve(reqs, realtime=False, keep_outputs=True)
    res_p, _ = PlainServer(bank).serve(reqs, realtime=False, keep_outputs=True)
    for r, rp in zip(res, res_p):
        q = r.request
        grid = smoe.make_grid(q.width, q.height, q.scale, q.origin_x, q.origin_y, mode="rbf")
        alone, _, _, _ = smoe.render(bank.rows(q.model), 3, 1, grid)
        assert torch.equal(r.image, alone) and torch.equal(rp.image, alone), q
