"""HIP-graph capture of fit steps: every replay must equal the same steps run eagerly,
bitwise, with eager work and synchronisations between replays; and the graphed loop must
survive a pair-capacity overflow (re-size, re-capture) with the same result."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _state(smoe, w, capacity=None, max_steps=64):
    import torch
    adam = smoe.AdamConfig(total_steps=2000)
    return smoe.FitState(torch.from_numpy(w.target).cuda(), torch.from_numpy(w.raw0).cuda(),
                         w.order, adam, max_steps=max_steps, capacity=capacity)


def test_graph_replays_equal_eager_steps():
    import torch

    import paper_2510_05814_amd as smoe
    print("[case] graph replay vs eager, 512^2 K=4096", flush=True)
    w = wl.workload(2)
    a = _state(smoe, w, capacity=400000)
    b = _state(smoe, w, capacity=400000)
    g = b.capture(6)
    assert b.steps_done() == 0  # capture runs nothing
    for r in range(4):
        for _ in range(6):
            a.step()
        b.replay(g)
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda")
        (junk * 2.0).sum().item()  # unrelated eager work between replays
        assert a.steps_done() == b.steps_done() == 6 * (r + 1)
        for name in ("raw", "m", "v", "model", "grads", "image", "denom"):
            assert torch.equal(getattr(a, name), getattr(b, name)), (r, name)
        assert torch.equal(a.losses(), b.losses())


def test_graphed_run_survives_overflow():
    import torch

    import paper_2510_05814_amd as smoe
    print("[case] graphed run with overflow", flush=True)
    w = wl.workload(1)
    a = _state(smoe, w, capacity=50000)
    b = _state(smoe, w, capacity=100)  # far too small: first replays are no-ops
    a.run(40)
    b.run_graphed(40, steps_per_graph=8, check_every=2)
    assert a.steps_done() == b.steps_done() == 40
    assert b.bins.capacity > 100
    assert torch.equal(a.raw, b.raw) and torch.equal(a.losses(), b.losses())
    h = b.losses().cpu().numpy()
    assert np.all(np.isfinite(h)) and h[-1] < h[0]
