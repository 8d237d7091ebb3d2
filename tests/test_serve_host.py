"""Host logic of the serving loop (no GPU): the pair bound that sizes a batch's workspace
never falls below the pairs the oracle's binning produces, and admission is FIFO, within
the budget and the batch limits."""
from collections import deque
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import workloads as wl
from paper_2510_05814_amd.serve import BoxSpans, admit


def test_pair_bound_covers_oracle_pairs():
    rng = np.random.default_rng(5)
    models = [wl.random_model(150, 3, 1, 48, 40, seed=300 + i, sig_lo=0.5, sig_hi=14.0)
              for i in range(3)]
    spans = BoxSpans(models, 3.0)
    ratios = []
    for _ in range(40):
        i = int(rng.integers(3))
        s = int(rng.integers(1, 5))
        W = int(rng.integers(1, 48 * s + 1))
        H = int(rng.integers(1, 40 * s + 1))
        ox = int(rng.integers(-20, 48 * s - W + 21))
        oy = int(rng.integers(-20, 40 * s - H + 21))
        P = oracle.bin(models[i].astype(np.float64), 3, 1, W, H, s, ox, oy)["P"]
        bound = spans.pair_bound(i, s, W, H)
        assert bound >= P, (i, s, W, H, ox, oy)
        if P:
            ratios.append(bound / P)
    # a bound, not a wild over-estimate, for windows that contain most kernels
    assert np.median(ratios) < 8.0


def test_pair_bound_single_kernel_closed_form():
    # one round kernel, l = 2: R = 6, a 12 px box overlaps <= 2 native blocks per axis, whose
    # 32 s sample points touch <= 2 s + 1 output blocks per axis
    m = np.zeros((1, 15), np.float64)
    m[0, 2] = m[0, 4] = 2.0
    spans = BoxSpans([m], 3.0)
    assert spans.pair_bound(0, 1, 256, 256) == 3 * 3
    assert spans.pair_bound(0, 1, 16, 256) == 2 * 3  # 16 px touch at most two blocks
    assert spans.pair_bound(0, 4, 256, 256) == 9 * 9
    for ox in range(16):
        P = oracle.bin(np.array([[8.0 + ox / 4, 8.0, 2.0, 0.0, 2.0, 0.0] + [0.5] * 9]), 3, 1,
                       64, 64)["P"]
        assert P <= 4


def test_pair_bound_with_sharpening_covers_oracle_pairs():
    """The box of a kernel sharpened by f has half-side R / f; the bound keyed by f covers
    the pairs of the sharpened model (L / f in binary32) at every factor, below and above 1."""
    rng = np.random.default_rng(6)
    models = [wl.random_model(120, 3, 1, 40, 36, seed=310 + i, sig_lo=0.5, sig_hi=12.0)
              for i in range(2)]
    spans = BoxSpans(models, 3.0)
    for _ in range(30):
        i = int(rng.integers(2))
        s = int(rng.integers(1, 4))
        f = float(rng.choice([0.6, 1.0, 1.3, 2.0, 3.7]))
        W, H = int(rng.integers(1, 40 * s + 1)), int(rng.integers(1, 36 * s + 1))
        ox, oy = int(rng.integers(-10, 11)), int(rng.integers(-10, 11))
        P = oracle.bin(oracle.sharpen(models[i], f), 3, 1, W, H, s, ox, oy)["P"]
        assert spans.pair_bound(i, s, W, H, f) >= P, (i, s, f, W, H, ox, oy)
    # sharpening shrinks the boxes: the bound does not grow with f
    assert spans.pair_bound(0, 2, 80, 72, 2.0) <= spans.pair_bound(0, 2, 80, 72)
    assert spans.pair_bound(0, 2, 80, 72, 0.0) == spans.pair_bound(0, 2, 80, 72, 1.0)


def _req(w, h):
    return SimpleNamespace(width=w, height=h)


def test_admit_fifo_budget_and_limits():
    fp = lambda b: sum(r.width * r.height for r in b)  # noqa: E731  bytes = pixels here
    q = deque([_req(10, 10), _req(20, 20), _req(5, 5), _req(1, 1)])
    got = admit(q, 0, 1000, fp, 8, 10 ** 9)
    assert [r.width for r in got] == [10, 20, 5, 1]   # 100 + 400 + 25 + 1 fits
    assert not q
    q = deque([_req(10, 10), _req(20, 20), _req(25, 25)])
    got = admit(q, 0, 1000, fp, 8, 10 ** 9)
    assert [r.width for r in got] == [10, 20]         # + 625 would exceed 1000
    q = deque([_req(10, 10), _req(31, 31), _req(1, 1)])
    got = admit(q, 0, 1000, fp, 8, 10 ** 9)
    assert [r.width for r in got] == [10]             # 31x31 does not fit: never skipped
    assert [r.width for r in q] == [31, 1]
    assert admit(q, 200, 1000, fp, 8, 10 ** 9) == []  # head waits for memory
    q = deque([_req(1, 1)] * 5)
    assert len(admit(q, 0, 1000, fp, 2, 10 ** 9)) == 2
    q = deque([_req(10, 10)] * 5)
    assert len(admit(q, 0, 10 ** 6, fp, 8, 250)) == 2  # pixel cap
    q = deque([_req(100, 100)])
    with pytest.raises(ValueError):
        admit(q, 0, 1000, fp, 8, 10 ** 9)


def test_window_layout_covers_every_pixel_h_times():
    """Block-overlapping windows (multi-model fusion): with displacement d every pixel lies
    in (16 / d)^2 windows, the windows stay inside the image and none is empty."""
    from paper_2510_05814_amd.multimodel import window_layout
    for (H, W) in [(16, 16), (37, 50), (64, 33)]:
        for d in (16, 8, 4, 2):
            cover = np.zeros((H, W), np.int64)
            for (y0, x0, h, w) in window_layout(H, W, d):
                assert 0 <= y0 and 0 <= x0 and h > 0 and w > 0 and y0 + h <= H and x0 + w <= W
                assert h <= 16 and w <= 16
                cover[y0:y0 + h, x0:x0 + w] += 1
            assert np.all(cover == (16 // d) ** 2), (H, W, d)
    with pytest.raises(ValueError):
        window_layout(16, 16, 3)


def test_model_bank_rejects_nonfinite_rows():
    import numpy as np
    import pytest as _pt

    from paper_2510_05814_amd.serve import ModelBank
    m = np.zeros((3, 15), np.float32)
    m[:, 2] = m[:, 4] = 1.0
    m[1, 7] = np.nan
    with _pt.raises(ValueError, match="model 0"):
        ModelBank([m], 3, 1, device="cpu")
