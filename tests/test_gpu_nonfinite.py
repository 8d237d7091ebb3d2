"""Kernel rows with NaN or infinite parameters: they take part nowhere -- the image, the
denominator and a fit of the other kernels are bitwise those without the rows -- and the
status words report them (smoe_read_status: SMOE_ERR_NONFINITE), per binning for a render and
from the step that meets them on for a fit."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

BAD = {7: (5, np.nan), 20: (10, np.inf), 33: (0, np.nan), 41: (4, -np.inf)}


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _poisoned(m):
    bad = m.copy()
    for j, (col, v) in BAD.items():
        bad[j, col] = v
    keep = np.array([j for j in range(m.shape[0]) if j not in BAD])
    return bad, m[keep]


@pytest.mark.parametrize("scale,ox,oy,trunc", [(1, 0, 0, "gradient"), (2, 5, -3, "gradient"),
                                               (3, 0, 7, "render")])
def test_nonfinite_rows_take_part_nowhere(scale, ox, oy, trunc):
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi as C
    say("nonfinite render", scale, ox, oy, trunc)
    W, H = 70, 52
    m = wl.random_model(60, 3, 1, W // scale + 2, H // scale + 2, seed=61)
    bad, kept = _poisoned(m)
    grid = smoe.make_grid(W, H, scale, ox, oy, trunc=trunc)
    img_b, D_b, _, b = smoe.render(dev(bad), 3, 1, grid)
    code, st = C.smoe_read_status(b.c, torch.cuda.current_stream().cuda_stream)
    assert code == C.SMOE_ERR_NONFINITE and st[3] == 1 and st[1] == 0
    img_k, D_k, _, bk = smoe.render(dev(kept), 3, 1, grid)
    assert torch.equal(img_b, img_k) and torch.equal(D_b, D_k)
    assert torch.isfinite(img_b).all()
    # the flag belongs to one binning: the same workspace with a finite model is clean
    smoe.bin(dev(m), 3, 1, grid, bins=b)
    code, st = C.smoe_read_status(b.c, torch.cuda.current_stream().cuda_stream)
    assert code == C.SMOE_OK and st[3] == 0
    # the static-workspace entry point reports it through status_out
    img_n, D_n, status = smoe.render_noalloc(dev(bad), 3, 1, grid)
    torch.cuda.synchronize()
    assert int(status[3]) == 1 and int(status[1]) == 0
    assert torch.equal(img_n, img_k)


def test_nonfinite_row_in_a_fit_is_inert():
    """A fit whose initial rows include non-finite ones: every other row, the Adam moments of
    those rows and the loss are bitwise those of fitting without them, and the status reports
    the rows after every step."""
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi as C
    say("nonfinite fit")
    w = wl.workload(2)
    H, W, Cc = w.target.shape
    raw = w.raw0.copy()
    bad, kept = _poisoned(raw)
    keep = [j for j in range(raw.shape[0]) if j not in BAD]
    adam = smoe.AdamConfig(total_steps=100)
    t = dev(w.target)
    sb = smoe.FitState(t, dev(bad), 1, adam, max_steps=6)
    sk = smoe.FitState(t, dev(kept), 1, adam, max_steps=6)
    for _ in range(3):
        sb.step()
        sk.step()
    torch.cuda.synchronize()
    assert torch.equal(sb.raw[keep], sk.raw)
    assert torch.equal(sb.m[keep], sk.m) and torch.equal(sb.v[keep], sk.v)
    assert torch.equal(sb.losses(), sk.losses())
    code, st = C.smoe_read_status(sb.bins.c, torch.cuda.current_stream().cuda_stream)
    assert code == C.SMOE_ERR_NONFINITE and st[3] == 1
    code, st = C.smoe_read_status(sk.bins.c, torch.cuda.current_stream().cuda_stream)
    assert code == C.SMOE_OK and st[3] == 0


def test_nan_target_pixel_is_reported_by_the_fit():
    """A NaN in the target makes the gradients of the kernels over that pixel NaN; Adam turns
    their rows non-finite and the status reports it after that step (the same fit on the
    clean target reports nothing)."""
    import torch

    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi as C
    say("nan target")
    w = wl.workload(1)
    tgt = w.target.copy()
    tgt[10, 20, 0] = np.nan
    st = smoe.FitState(dev(tgt), dev(w.raw0), w.order, smoe.AdamConfig.constant(1e-2, 10),
                       max_steps=4)
    clean = smoe.FitState(dev(w.target), dev(w.raw0), w.order,
                          smoe.AdamConfig.constant(1e-2, 10), max_steps=4)
    for f in (st, clean):
        f.step()
    code, s = C.smoe_read_status(st.bins.c, torch.cuda.current_stream().cuda_stream)
    assert code == C.SMOE_ERR_NONFINITE and s[3] == 1
    assert not torch.isfinite(st.raw).all()
    code, s = C.smoe_read_status(clean.bins.c, torch.cuda.current_stream().cuda_stream)
    assert code == C.SMOE_OK and s[3] == 0
