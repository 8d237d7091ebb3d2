"""Pins of the oracle's multi-model estimator (Sec. V-C, Eq. (10)-(11)) against what the
definition fixes: every pixel is covered by (window/d)^2 windows; identical hypotheses
average to the hypothesis itself; window models of known constant values average to a closed
form of the pixel position.  Planted mistakes in the estimator (its window placement and its
average) must each fail one of these pins."""
import inspect
import textwrap

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("H,W,d,window", [(40, 37, 8, 16), (16, 16, 16, 16), (33, 50, 4, 16),
                                          (21, 18, 2, 16), (5, 7, 4, 16), (29, 31, 4, 12)])
def test_every_pixel_has_the_same_number_of_windows(H, W, d, window):
    m = window // d
    rects = oracle.window_rects(H, W, d, window)
    if H >= window and W >= window:
        assert len(set(rects)) == len(rects)
    cnt = np.zeros((H, W), np.int64)
    for (y0, x0, h, w) in rects:
        assert 0 <= y0 and 0 <= x0 and 1 <= h <= window and 1 <= w <= window
        assert y0 + h <= H and x0 + w <= W
        cnt[y0:y0 + h, x0:x0 + w] += 1
    assert np.all(cnt == m * m)


def _global_model(rng, K, H, W):
    """Random kernels with centres on a 1/64 grid, so that the translation into any window's
    coordinates is exact in binary32."""
    mu = np.stack([np.floor(rng.uniform(-4, W + 4, K) * 64) / 64,
                   np.floor(rng.uniform(-4, H + 4, K) * 64) / 64], 1)
    l11 = rng.uniform(1.5, 5.0, K)
    l22 = rng.uniform(1.5, 5.0, K)
    l21 = rng.uniform(-2.0, 2.0, K)
    rho = rng.uniform(-1.0, 1.0, K)
    experts = rng.uniform(0.0, 1.0, (K, 9))
    return np.column_stack([mu, l11, l21, l22, rho, experts])


def _translated(model, x0, y0):
    m = model.copy()
    m[:, 0] -= x0
    m[:, 1] -= y0
    return m


@pytest.mark.parametrize("d", [16, 8, 4])
def test_identical_hypotheses_average_to_the_hypothesis(d):
    """Every window holds the whole global model, moved into its own coordinates.  With the
    ellipse test deciding (the render's value is then a function of the point alone) every
    window predicts the global render at each of its pixels, and the mean of equal values is
    that value."""
    rng = np.random.default_rng(d)
    H, W = 37, 45
    g = _global_model(rng, 30, H, W)
    models = [_translated(g, x0, y0) for (y0, x0, _, _) in oracle.window_rects(H, W, d)]
    fused = oracle.fuse_windows(models, 3, 1, H, W, d, trunc="render")
    y, _ = oracle.render(g, 3, 1, W, H, trunc="render")
    assert np.max(np.abs(fused - y)) <= 1e-12


def _constant_window_models(H, W, d, window=16):
    """Window (ky, kx) -- counted from the window whose span ends d pixels into the image --
    predicts the constant kx + 100 ky everywhere in it (one broad kernel with a constant
    expert; C = 1, order 0)."""
    models = []
    for (y0, x0, h, w) in oracle.window_rects(H, W, d, window):
        # unclipped start: the clipped start if the window begins inside the image, else
        # `window` pixels before its end (the images are at least a window wide here)
        sx = x0 if x0 > 0 else x0 + w - window
        sy = y0 if y0 > 0 else y0 + h - window
        kx, ky = (sx + window) // d - 1, (sy + window) // d - 1
        models.append(np.array([[w / 2, h / 2, 100.0, 0.0, 100.0, 0.0, kx + 100.0 * ky]]))
    return models


@pytest.mark.parametrize("H,W,d,window", [(40, 37, 8, 16), (16, 16, 16, 16), (33, 50, 4, 16),
                                          (20, 18, 2, 16), (29, 31, 4, 12)])
def test_constant_hypotheses_average_in_closed_form(H, W, d, window):
    """The windows covering pixel x along an axis are k = floor(x/d) ... floor(x/d) + m - 1
    (m = window/d), so the mean of the window indices is floor(x/d) + (m - 1)/2."""
    m = window // d
    fused = oracle.fuse_windows(_constant_window_models(H, W, d, window), 1, 0, H, W, d,
                                window)
    ys, xs = np.mgrid[0:H, 0:W]
    want = (xs // d + (m - 1) / 2) + 100.0 * (ys // d + (m - 1) / 2)
    assert np.max(np.abs(fused[..., 0] - want)) <= 1e-9


# Planted mistakes in the estimator: (label, original text, planted text)
FUSION_MUTANTS = [
    ("first window starts a whole window before the image",
     "range(-(window - d), n, d)", "range(-window, n, d)"),
    ("windows stop one displacement early", "range(-(window - d), n, d)",
     "range(-(window - d), n - d, d)"),
    ("window rows and columns swapped in the placement",
     "acc[y0:y0 + h, x0:x0 + w] += y", "acc[x0:x0 + w, y0:y0 + h] += y.transpose(1, 0, 2)"),
    ("sum instead of mean", "return acc / cnt[..., None]", "return acc"),
    ("clipped windows keep their unclipped start", "out.append((cover[0], len(cover)))",
     "out.append((start, len(cover)))"),
    ("windows clipped on the left only", "p for p in range(start, start + window) if 0 <= p < n",
     "p for p in range(start, start + window) if 0 <= p"),
    ("window models rendered one pixel shifted", "render(model, C, order, w, h,",
     "render(model, C, order, w, h, ox=1,"),
    ("models paired with the windows in reverse order", "zip(rects, models)",
     "zip(rects, models[::-1])"),
]


def _mutated(fn, old, new):
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, old
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns[fn.__name__], ns


@pytest.mark.parametrize("label,old,new", FUSION_MUTANTS, ids=[m[0] for m in FUSION_MUTANTS])
def test_planted_fusion_mistakes_fail_a_pin(monkeypatch, label, old, new):
    fn = oracle.window_rects if ("range(" in old or "append" in old) else oracle.fuse_windows
    mut, _ = _mutated(fn, old, new)
    monkeypatch.setattr(oracle, fn.__name__, mut)
    if fn is oracle.fuse_windows:
        # fuse_windows looks window_rects up in the module namespace: keep the real one
        mut.__globals__["window_rects"] = oracle.window_rects
    pinned = [lambda: test_every_pixel_has_the_same_number_of_windows(40, 37, 8, 16),
              lambda: test_every_pixel_has_the_same_number_of_windows(21, 18, 2, 16),
              lambda: test_identical_hypotheses_average_to_the_hypothesis(8),
              lambda: test_constant_hypotheses_average_in_closed_form(40, 37, 8, 16),
              lambda: test_constant_hypotheses_average_in_closed_form(33, 50, 4, 16)]
    failed = 0
    for pin in pinned:
        try:
            pin()
        except Exception:  # noqa: BLE001 -- an assertion or an indexing error both fail the pin
            failed += 1
    assert failed, f"planted mistake not caught: {label}"
