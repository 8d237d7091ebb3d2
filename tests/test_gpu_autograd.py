"""The autograd.Function path: gradients against the FP64 oracle and against the fused fit
step; it composes with torch optimizers and upstream gradients of any loss."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _groups(C, order):
    g = {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5], "a": list(range(6, 6 + C))}
    if order == 1:
        g["wx"] = list(range(6 + C, 6 + 2 * C))
        g["wy"] = list(range(6 + 2 * C, 6 + 3 * C))
    return g


def _group_err(g, g_ref, C, order):
    """Largest error over a parameter group relative to that group's largest oracle value."""
    return max(float(np.max(np.abs(g[:, c] - g_ref[:, c])) / max(np.max(np.abs(g_ref[:, c])), 1e-300))
               for c in _groups(C, order).values())


def test_autograd_mse_gradient_matches_oracle(record_error):
    import torch

    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd vs oracle, crop", flush=True)
    tgt, raw = wl.fd_crop_case(seed=17)
    H, W, C = tgt.shape
    r = _dev(raw).requires_grad_(True)
    img = smoe_render(r, C, 1, W, H)
    loss = torch.mean((img - _dev(tgt)) ** 2)
    loss.backward()
    model = oracle.materialize(raw.astype(np.float64), C, 1)
    l_o, g_o = oracle.loss_grad(model, C, 1, W, H, target=tgt, trunc="render")
    g = r.grad.cpu().numpy()
    assert abs(loss.item() - l_o) <= 1e-5 * l_o
    err = _group_err(g, g_o, C, 1)
    record_error("autograd grad rel (per group)", err, 1e-3)
    assert err <= 1e-3


def test_autograd_default_is_the_forward_derivative(record_error):
    """With the default reading the backward is the derivative of the forward: central
    differences of the autograd forward's own loss (FP64 oracle forward at the perturbed
    parameters, h = 1e-6, on the crop whose pairs keep clear of the truncation edge) match the
    GPU gradient per group."""
    import torch

    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd default vs central differences", flush=True)
    tgt, raw = wl.fd_crop_case()
    H, W, C = tgt.shape
    raw = raw.astype(np.float64)
    r = _dev(raw).requires_grad_(True)
    torch.mean((smoe_render(r, C, 1, W, H) - _dev(tgt)) ** 2).backward()
    h = 1e-6
    fd = np.zeros_like(raw)
    for j in range(raw.shape[0]):
        for k in range(raw.shape[1]):
            rp, rm = raw.copy(), raw.copy()
            rp[j, k] += h
            rm[j, k] -= h
            yp, _ = oracle.render(oracle.materialize(rp, C, 1), C, 1, W, H, trunc="render")
            ym, _ = oracle.render(oracle.materialize(rm, C, 1), C, 1, W, H, trunc="render")
            fd[j, k] = (np.mean((yp - tgt) ** 2) - np.mean((ym - tgt) ** 2)) / (2 * h)
    err = _group_err(r.grad.cpu().numpy(), fd, C, 1)
    record_error("autograd default grad vs central differences (per group)", err, 1e-3)
    assert err <= 1e-3


def test_autograd_full_size_against_oracle(record_error):
    """SMoERender forward + backward at 2048^2 RGB, K = 65536 linear experts (perturbed from
    the grid init), MSE to the denoising target: the whole image and the loss against the FP64
    oracle's full render, and the gradients of 24 sampled kernels per parameter group."""
    import torch

    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd 2048^2 K=65536", flush=True)
    w = wl.workload(3)
    H, W, C = w.target.shape
    rng = np.random.default_rng(23)
    raw = w.raw0.astype(np.float64)
    raw[:, :2] += rng.uniform(-2, 2, (w.K, 2))
    raw[:, 3] = rng.uniform(-1, 1, w.K)
    raw[:, 9:] = rng.uniform(-0.01, 0.01, (w.K, 6))
    raw = raw.astype(np.float32)
    r = _dev(raw).requires_grad_(True)
    img = smoe_render(r, C, 1, W, H)
    loss = torch.mean((img - _dev(w.target)) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    model = oracle.materialize(raw.astype(np.float64), C, 1)
    y_o, _ = oracle.render(model, C, 1, W, H, trunc="render")
    ey = float(np.max(np.abs(img.detach().cpu().numpy() - y_o)))
    record_error("autograd 2048 full image abs", ey, 1e-5)
    assert ey <= 1e-5
    l_o = float(np.mean((y_o - w.target) ** 2))
    el = abs(loss.item() - l_o) / l_o
    record_error("autograd 2048 loss rel", el, 1e-5)
    assert el <= 1e-5
    sel = np.concatenate([[0, w.K - 1, 255, w.K - 256], rng.choice(w.K, 20, replace=False)])
    _, g_o = oracle.loss_grad(model, C, 1, W, H, target=w.target, kernels=sel, trunc="render")
    err = _group_err(r.grad.cpu().numpy()[sel], g_o, C, 1)
    record_error("autograd 2048 sampled grad rel (per group)", err, 1e-3)
    assert err <= 1e-3


def test_autograd_arbitrary_upstream_gradient(record_error):
    """A non-MSE loss: L = sum(weights * image) -> upstream gradient = weights."""
    import torch

    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd upstream", flush=True)
    W, H = 41, 35
    m = wl.random_model(60, 3, 1, W, H, seed=91)
    raw = m.astype(np.float64).copy()
    raw[:, 2] = np.log(raw[:, 2])
    raw[:, 4] = np.log(raw[:, 4])
    wts = np.random.default_rng(2).normal(size=(H, W, 3))
    r = _dev(raw).requires_grad_(True)
    (smoe_render(r, 3, 1, W, H) * _dev(wts)).sum().backward()
    _, g_o = oracle.loss_grad(oracle.materialize(raw, 3, 1), 3, 1, W, H, grad_y=wts,
                              trunc="render")
    err = _group_err(r.grad.cpu().numpy(), g_o, 3, 1)
    record_error("autograd upstream grad rel", err, 1e-3)
    assert err <= 1e-3


def test_autograd_equals_fused_fit_step_gradient(record_error):
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd vs fit step", flush=True)
    w = wl.workload(2)
    H, W, C = w.target.shape
    t = _dev(w.target)
    st = smoe.FitState(t, _dev(w.raw0), 1, smoe.AdamConfig(total_steps=100), max_steps=2)
    st.step()
    r = _dev(w.raw0).requires_grad_(True)
    loss = torch.mean((smoe_render(r, C, 1, W, H, trunc="gradient") - t) ** 2)
    loss.backward()
    err = _group_err(r.grad.cpu().numpy(), st.grads.cpu().numpy(), C, 1)
    record_error("autograd vs fused fit-step grad rel (per group)", err, 1e-5)
    assert err <= 1e-5
    assert abs(loss.item() - st.losses()[0].item()) <= 1e-6 * loss.item()


def test_autograd_with_torch_adam_reduces_loss():
    import torch

    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd + torch.optim.Adam", flush=True)
    w = wl.workload(1)
    H, W, C = w.target.shape
    t = _dev(w.target)
    r = _dev(w.raw0).requires_grad_(True)
    opt = torch.optim.Adam([r], lr=1e-2)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = torch.mean((smoe_render(r, C, 0, W, H) - t) ** 2)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert losses[-1] < 0.8 * losses[0]


@pytest.mark.parametrize("mode,trunc", [("rbf", "gradient"), ("smoe", "gradient"), ("rbf", "render")])
def test_autograd_modes_against_oracle(mode, trunc, record_error):
    """The autograd path with the RBF sum of Eq. (1) and/or the ellipse test in the render."""
    import torch

    from paper_2510_05814_amd.autograd import smoe_render
    print("[case] autograd", mode, trunc, flush=True)
    W, H = 44, 37
    m = wl.random_model(70, 3, 1, W, H, seed=93, rho_std=0.3)
    m[:, 5] -= 1.0
    raw = m.astype(np.float64).copy()
    raw[:, 2] = np.log(raw[:, 2])
    raw[:, 4] = np.log(raw[:, 4])
    wts = np.random.default_rng(4).normal(size=(H, W, 3))
    r = _dev(raw).requires_grad_(True)
    img = smoe_render(r, 3, 1, W, H, mode=mode, trunc=trunc)
    (img * _dev(wts)).sum().backward()
    model = oracle.materialize(raw, 3, 1)
    y_o, _ = oracle.render(model, 3, 1, W, H, rbf=(mode == "rbf"), trunc=trunc)
    ey = float(np.max(np.abs(img.detach().cpu().numpy() - y_o))) / max(1.0, float(np.abs(y_o).max()))
    _, g_o = oracle.loss_grad(model, 3, 1, W, H, grad_y=wts, rbf=(mode == "rbf"), trunc=trunc)
    err = _group_err(r.grad.cpu().numpy(), g_o, 3, 1)
    record_error(f"autograd {mode}/{trunc} image", ey, 1e-5)
    record_error(f"autograd {mode}/{trunc} grad rel", err, 1e-3)
    assert ey <= 1e-5 and err <= 1e-3
