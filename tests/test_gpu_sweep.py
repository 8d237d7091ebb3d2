"""A seeded sweep over the rule's settings and the model shapes: for each of 40 random small
cases (channels, expert order, regression mode, truncation reading, box, sharpening factor,
scale, origin, raster and model size), the block lists bit-exact against the oracle's, the
image within 1e-5 of the peak magnitude, and -- where the backward applies (no sharpening) --
the gradient within 1e-3 of the largest oracle gradient of each parameter group."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _cases(n=40, seed=900):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        out.append(dict(
            C=int(rng.choice([1, 3])), order=int(rng.integers(0, 2)),
            mode=str(rng.choice(["smoe", "rbf"])), trunc=str(rng.choice(["gradient", "render"])),
            box=str(rng.choice(["square", "tight"])),
            sharpen=float(rng.choice([1.0, 1.0, 0.8, 1.6])), s=int(rng.integers(1, 4)),
            W=int(rng.integers(1, 70)), H=int(rng.integers(1, 60)), K=int(rng.integers(0, 120)),
            seed=seed + i))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[f"case{i}" for i in range(len(CASES))])
def test_sweep_against_oracle(case, record_error):
    import torch

    import paper_2510_05814_amd as smoe
    print("[case] sweep", case, flush=True)
    C, order, mode, trunc = case["C"], case["order"], case["mode"], case["trunc"]
    box, f, s, W, H, K = case["box"], case["sharpen"], case["s"], case["W"], case["H"], case["K"]
    rng = np.random.default_rng(case["seed"])
    ox, oy = int(rng.integers(0, s)), int(rng.integers(0, s))
    OW, OH = max(1, s * W - ox), max(1, s * H - oy)
    m_np = wl.stretched_model(K, C, order, W, H, case["seed"]) if K else \
        np.zeros((0, wl.num_params(C, order)), np.float32)
    if K and mode == "rbf":
        m_np[:, 5] -= 1.0
    m = torch.from_numpy(np.ascontiguousarray(m_np)).cuda()
    grid = smoe.make_grid(OW, OH, s, ox, oy, sharpen=f, box=box, mode=mode, trunc=trunc)
    b = smoe.bin(m, C, order, grid)
    over, st = b.read_status()
    assert not over
    ms = oracle.sharpen(m_np.astype(np.float64), f)
    boxi = 1 if box == "tight" else 0
    ob = oracle.bin(ms, C, order, OW, OH, s, ox, oy, box=boxi, trunc=trunc)
    P = st[0]
    assert P == ob["P"]
    assert np.array_equal(b.tile_rects().cpu().numpy(), ob["tile_rects"])
    assert np.array_equal(b.vals(P).cpu().numpy().view(np.uint32), ob["vals"])
    assert np.array_equal(b.ranges(smoe.tiles(OW, OH, ox, oy)).cpu().numpy(), ob["ranges"])
    t_np = rng.uniform(0, 1, (OH, OW, C)).astype(np.float32)
    t = torch.from_numpy(t_np).cuda()
    img, D, loss, b = smoe.render(m, C, order, grid, bins=b, target=t)
    y_o, _ = oracle.render(ms, C, order, OW, OH, s, ox, oy, box=boxi, rbf=(mode == "rbf"),
                           trunc=trunc)
    peak = max(1.0, float(np.abs(y_o).max()) if y_o.size else 1.0)
    ey = float(np.max(np.abs(img.cpu().numpy() - y_o))) / peak
    record_error("sweep image / peak", ey, 1e-5)
    assert ey <= 1e-5
    if f != 1.0 or K == 0:
        return
    g = smoe.render_backward(m, C, order, grid, b, img, D, target=t).cpu().numpy()
    _, g_o = oracle.loss_grad(ms, C, order, OW, OH, target=t_np, s=s, ox=ox, oy=oy, box=boxi,
                              rbf=(mode == "rbf"), trunc=trunc)
    groups = [[0, 1], [2], [3], [4], [5], list(range(6, 6 + C))]
    if order == 1:
        groups += [list(range(6 + C, 6 + 2 * C)), list(range(6 + 2 * C, 6 + 3 * C))]
    for cols in groups:
        scale = float(np.max(np.abs(g_o[:, cols])))
        if scale == 0:
            assert np.max(np.abs(g[:, cols])) == 0
            continue
        e = float(np.max(np.abs(g[:, cols] - g_o[:, cols]))) / scale
        record_error(f"sweep grad cols {cols[0]} rel", e, 1e-3)
        assert e <= 1e-3, (cols, e)
