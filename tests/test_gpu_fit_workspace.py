"""A fresh fit on a workspace holding arbitrary bytes: the first step clears the status
words (overflow flags included) itself, so the fit proceeds exactly as on a zeroed
workspace."""
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def test_fresh_fit_on_dirty_workspace():
    import paper_2510_05814_amd as smoe

    w = wl.workload(1)
    target = torch.from_numpy(w.target).cuda()
    raw0 = torch.from_numpy(w.raw0).cuda()
    adam = smoe.AdamConfig.constant(1e-2, 20)
    print("[case] fit 64x64 K=64 on a zeroed and on a 0xFF-filled workspace", flush=True)
    a = smoe.FitState(target, raw0, w.order, adam, max_steps=20)
    b = smoe.FitState(target, raw0, w.order, adam, max_steps=20)
    b.bins.ws.fill_(0xFF)
    for _ in range(20):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert a.steps_done() == b.steps_done() == 20
    assert torch.equal(a.raw, b.raw)
    assert torch.equal(a.losses(), b.losses())
    over, _ = b.bins.read_status()
    assert not over


def test_steps_without_render_output_are_bitwise_the_same():
    """write_render = 0 skips only the stores of image and denom: losses, gradients and
    parameters are bitwise those of steps that store them, and image / denom are untouched."""
    import paper_2510_05814_amd as smoe

    w = wl.workload(2)
    target = torch.from_numpy(w.target).cuda()
    raw0 = torch.from_numpy(w.raw0).cuda()
    adam = smoe.AdamConfig(total_steps=100)
    print("[case] fit 512^2 with and without render output", flush=True)
    a = smoe.FitState(target, raw0, w.order, adam, max_steps=8)
    b = smoe.FitState(target, raw0, w.order, adam, max_steps=8, write_render=False)
    b.image.fill_(-1.0)
    b.denom.fill_(-1.0)
    for _ in range(6):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert torch.equal(a.raw, b.raw) and torch.equal(a.grads, b.grads)
    assert torch.equal(a.losses(), b.losses())
    assert bool((b.image == -1.0).all()) and bool((b.denom == -1.0).all())
    b.set_write_render(True)
    a.step()
    b.step()
    torch.cuda.synchronize()
    assert torch.equal(a.image, b.image) and torch.equal(a.denom, b.denom)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_bucket_width_does_not_change_the_fit(n):
    """The fit step's bucket width (pair capacity / blocks) moves where entries and partial
    rows are stored, never the sorted lists or any summation order: fits with 64- and
    96-entry buckets are bitwise the same."""
    import paper_2510_05814_amd as smoe

    w = wl.workload(n)
    H, W, _ = w.target.shape
    target = torch.from_numpy(w.target).cuda()
    raw0 = torch.from_numpy(w.raw0).cuda()
    adam = smoe.AdamConfig(total_steps=1000)
    T = smoe.tiles(W, H)
    print(f"[case] bucket widths 64 and 96, workload {n}", flush=True)
    a = smoe.FitState(target, raw0, w.order, adam, max_steps=8, capacity=T * 64)
    b = smoe.FitState(target, raw0, w.order, adam, max_steps=8, capacity=T * 96)
    for _ in range(8):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert not a.bins.read_status()[0] and not b.bins.read_status()[0]
    assert torch.equal(a.raw, b.raw) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
    assert torch.equal(a.grads, b.grads)
    assert torch.equal(a.losses(), b.losses())
    assert torch.equal(a.image, b.image)
