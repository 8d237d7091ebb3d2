"""smoe_render_noalloc (the entry point for callers that cannot allocate device memory)
against smoe_bin + smoe_render with a caller workspace: bitwise equal images and
denominators, and the same status words, on two calls in a row (the second on a smaller
raster and model, so that it runs over the contents the first left in the static
workspace)."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _case(smoe, K, C, order, W, H, seed, **grid_kw):
    import torch

    model = torch.from_numpy(wl.random_model(K, C, order, W, H, seed).astype(np.float32)).cuda()
    g = smoe.make_grid(W, H, **grid_kw)
    print(f"[case] noalloc K={K} C={C} order={order} {W}x{H} {grid_kw}", flush=True)
    img_ref, den_ref, _, bins = smoe.render(model, C, order, g)
    _, st_ref = bins.read_status()
    img, den, status = smoe.render_noalloc(model, C, order, g)
    torch.cuda.synchronize()
    assert torch.equal(img, img_ref)
    assert torch.equal(den, den_ref)
    st = status.cpu().tolist()
    assert st[1] == 0 and st[0] == st_ref[0] and st[2] == st_ref[2], (st, st_ref)
    return img


def test_noalloc_equals_workspace_render_twice():
    import paper_2510_05814_amd as smoe

    a = _case(smoe, 900, 3, 1, 203, 171, 11, scale=2, origin_x=5, origin_y=3)
    b = _case(smoe, 120, 1, 0, 37, 29, 12)
    assert a.shape != b.shape


def test_noalloc_preallocated_outputs_and_limits():
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi as C

    K, Cc, order, W, H = 300, 3, 1, 64, 48
    model = torch.from_numpy(wl.random_model(K, Cc, order, W, H, 5).astype(np.float32)).cuda()
    g = smoe.make_grid(W, H)
    img = torch.full((H, W, Cc), 7.0, device="cuda")
    den = torch.full((H, W), 7.0, device="cuda")
    st = torch.full((4,), 9, dtype=torch.int32, device="cuda")
    smoe.render_noalloc(model, Cc, order, g, img, den, st)
    ref, dref, _, _ = smoe.render(model, Cc, order, g)
    torch.cuda.synchronize()
    assert torch.equal(img, ref) and torch.equal(den, dref)
    assert st[1].item() == 0
    # a model whose per-kernel arrays alone exceed the static workspace is rejected before
    # any launch
    big = torch.zeros((1 << 20, 15), dtype=torch.float32, device="cuda")
    with pytest.raises(C.SmoeError) as e:
        smoe.render_noalloc(big, 3, 1, g)
    assert e.value.code == C.SMOE_ERR_TOO_LARGE
