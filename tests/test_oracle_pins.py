"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

None of these tests compares the oracle with itself or with the GPU path.  Each
one checks a value against an independent route to it: a library routine
(numpy.linalg, scipy.special.softmax, torch.optim.Adam), a closed form, brute
force on tiny inputs, an invariant of the model, or central finite differences.
A dropped term, a sign error, a swapped axis or a transposed operand anywhere in
the oracle makes at least one of them fail (see test_planted_mistakes_are_caught).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

R = 3.0


def sigma_of(model):
    """Covariances Sigma = L L^T from materialized rows."""
    L = np.zeros((model.shape[0], 2, 2))
    L[:, 0, 0] = model[:, 2]
    L[:, 1, 0] = model[:, 3]
    L[:, 1, 1] = model[:, 4]
    return L @ np.transpose(L, (0, 2, 1))


def maha_np(model, xs, ys):
    """(x-mu)^T Sigma^-1 (x-mu) for every kernel and point, via numpy.linalg.solve."""
    S = sigma_of(model.astype(np.float64))
    d = np.stack([xs[None, :] - model[:, 0:1].astype(np.float64),
                  ys[None, :] - model[:, 1:2].astype(np.float64)], axis=1)  # [K, 2, n]
    sol = np.linalg.solve(S, d)
    return np.einsum("kin,kin->kn", d, sol)


def centres(W, H):
    v, u = np.mgrid[0:H, 0:W]
    return u.ravel(), v.ravel(), u.ravel() + 0.5, v.ravel() + 0.5


# --------------------------------------------------------------------------- geometry


def test_denominator_is_pi_times_gaussian_eq2_eq4():
    """D(x) = sum_j pi_j K_j(x) (Eq. 2, 4): one kernel at a time, untruncated, against
    the Mahalanobis form computed by numpy.linalg.solve on Sigma = L L^T."""
    W, H = 23, 19
    m = wl.random_model(6, 1, 0, W, H, seed=11, margin=0.0)
    u, v, x, y = centres(W, H)
    q = maha_np(m, x, y)
    for j in range(m.shape[0]):
        _, D = oracle.render(m[j:j + 1], 1, 0, W, H, truncated=False)
        ref = np.exp(m[j, 5].astype(np.float64) - 0.5 * q[j]).reshape(H, W)
        np.testing.assert_allclose(D, ref, rtol=1e-12, atol=0)


def test_hand_computed_single_kernel():
    """Closed form by hand: mu = (8, 8), L = 4 I, rho = 0.  Pixel (11, 7) has its centre at
    (11.5, 7.5): q = (3.5^2 + 0.5^2)/16 = 0.78125, so D = exp(-0.390625)."""
    m = np.array([[8.0, 8.0, 4.0, 0.0, 4.0, 0.0, 0.25]])
    y, D = oracle.render(m, 1, 0, 16, 16, pixels=[(11, 7)])
    assert D[0] == pytest.approx(math.exp(-0.390625), rel=1e-15)
    assert y[0, 0] == pytest.approx(0.25, rel=1e-15)
    # pixel (14, 8): centre (14.5, 8.5), q = (6.5^2 + 0.5^2)/16 = 2.65625 -> inside r = 3
    # pixel (8, 0):  centre (8.5, 0.5),  q = (0.25 + 56.25)/16 = 3.53125 -> inside
    # pixel (0, 0):  q = (56.25 + 56.25)/16 = 7.03125 -> inside;  r = 2.5 excludes it
    _, D2 = oracle.render(m, 1, 0, 16, 16, pixels=[(14, 8), (8, 0), (0, 0)])
    np.testing.assert_allclose(D2, np.exp(-0.5 * np.array([2.65625, 3.53125, 7.03125])), rtol=1e-15)
    _, D3 = oracle.render(m, 1, 0, 16, 16, pixels=[(0, 0)], r=2.5, trunc="render")
    assert D3[0] == 0.0
    # with the ellipse in the gradient only, the kernel's box (half-side 10) still covers
    # block 0, so pixel (0, 0) keeps its term
    _, D4 = oracle.render(m, 1, 0, 16, 16, pixels=[(0, 0)], r=2.5)
    assert D4[0] == pytest.approx(math.exp(-0.5 * 7.03125), rel=1e-15)


def _np_native_blocks(lo, hi):
    """Native 16x16 blocks [b0, b1] of the native pixel centres c + 0.5 in [lo, hi] (FP64), or
    None."""
    c0, c1 = int(np.ceil(lo - 0.5)), int(np.floor(hi - 0.5))
    return (c0 >> 4, c1 >> 4) if c0 <= c1 else None


def _np_output_blocks(blocks, n, s=1, o=0):
    """The output blocks (first, last) of an axis of n points sampled at ((o + u) + 0.5) / s
    whose native block floor(x / 16) lies in `blocks` -- output blocks of 16 aligned to
    multiples of 16 in o + u, numbered from the one holding the first point -- and the native
    blocks clamped to those the points reach, by brute force over every point; None if no
    point is in them."""
    if blocks is None:
        return None
    nb = np.floor((np.arange(n) + o + 0.5) / s / 16).astype(np.int64)
    hit = np.nonzero((nb >= blocks[0]) & (nb <= blocks[1]))[0]
    if hit.size == 0:
        return None
    first = (o + hit[0]) // 16 - o // 16, (o + hit[-1]) // 16 - o // 16
    return first, (max(blocks[0], nb[0]), min(blocks[1], nb[-1]))


def test_box_half_side_is_r_sqrt_lambda_max():
    """The square box of Fig. 3b has half-side r*sqrt(lambda_max(Sigma)); a kernel's native
    blocks are those of the native pixel centres inside it (eigvalsh in FP64), the raster's
    output blocks are those of its sample points in them -- except where a centre sits within
    1e-3 px of an edge (binary32 rounding may go either way there)."""
    W, H = 97, 83
    m = wl.random_model(400, 1, 0, W, H, seed=12)
    lam = np.linalg.eigvalsh(sigma_of(m.astype(np.float64)))[:, -1]
    Rh = R * np.sqrt(lam)
    checked = 0
    for (s, ox, oy) in [(1, 0, 0), (1, 5, 9), (3, 7, 2)]:
        Wo, Ho = s * W - ox, s * H - oy
        b = oracle.bin(m, 1, 0, Wo, Ho, s, ox, oy)
        for j in range(m.shape[0]):
            lo_x, hi_x = m[j, 0] - Rh[j], m[j, 0] + Rh[j]
            lo_y, hi_y = m[j, 1] - Rh[j], m[j, 1] + Rh[j]
            edges = np.array([lo_x, hi_x, lo_y, hi_y]) - 0.5
            if np.min(np.abs(edges - np.round(edges))) < 1e-3:
                continue
            ax = _np_output_blocks(_np_native_blocks(lo_x, hi_x), Wo, s, ox)
            ay = _np_output_blocks(_np_native_blocks(lo_y, hi_y), Ho, s, oy)
            if ax is None or ay is None:
                assert b["counts"][j] == 0, j
                assert list(b["tile_rects"][j]) == [0, 0, -1, -1]
                assert list(b["native_rects"][j]) == [0, 0, -1, -1]
            else:
                (tx, nx), (ty, ny) = ax, ay
                assert list(b["tile_rects"][j]) == [tx[0], ty[0], tx[1], ty[1]], (s, j)
                assert list(b["native_rects"][j]) == [nx[0], ny[0], nx[1], ny[1]], (s, j)
                assert b["counts"][j] == (tx[1] - tx[0] + 1) * (ty[1] - ty[0] + 1)
            checked += 1
    assert checked > 1000


def test_box_contains_ellipse_boundary():
    """Every point of the r-ellipse boundary lies in the square box (Sec. IV-B): 10^4
    boundary points per kernel, mu + r L (cos t, sin t)."""
    m = wl.random_model(200, 1, 0, 400, 400, seed=13, sig_lo=0.5, sig_hi=40.0, margin=0.0)
    lam = np.linalg.eigvalsh(sigma_of(m.astype(np.float64)))[:, -1]
    t = np.linspace(0, 2 * np.pi, 10000, endpoint=False)
    circ = np.stack([np.cos(t), np.sin(t)])
    for j in range(m.shape[0]):
        Lj = np.array([[m[j, 2], 0.0], [m[j, 3], m[j, 4]]], dtype=np.float64)
        pts = R * (Lj @ circ)
        assert np.max(np.abs(pts)) <= R * math.sqrt(lam[j]) * (1 + 1e-12)


def test_truncation_rule_matches_ellipse_and_stays_in_box():
    """Brute force over every pixel, one kernel at a time: the oracle's participation set
    {D > 0} equals {q <= r^2} (numpy FP64) away from a 1e-5 band, and lies inside the
    kernel's native blocks, so the block conjunct of the rule never removes a pixel."""
    W, H = 61, 45
    m = wl.random_model(60, 1, 0, W, H, seed=14, sig_lo=0.7, sig_hi=8.0)
    u, v, x, y = centres(W, H)
    q = maha_np(m, x, y)
    b = oracle.bin(m, 1, 0, W, H)
    for j in range(m.shape[0]):
        _, D = oracle.render(m[j:j + 1], 1, 0, W, H, trunc="render")
        on = D.ravel() > 0
        band = np.abs(q[j] - R * R) < 1e-5
        assert np.array_equal(on[~band], (q[j] <= R * R)[~band]), j
        nr = b["native_rects"][j]
        bu, bv = u[on] >> 4, v[on] >> 4
        assert np.all((bu >= nr[0]) & (bu <= nr[2]) & (bv >= nr[1]) & (bv <= nr[3]))


def test_bins_bruteforce_tiny():
    """Block lists (Sec. IV-C) against a tile x kernel double loop, and the pair order
    against Python's sort of (block, kernel) tuples."""
    for (W, H, K, seed) in [(33, 47, 30, 21), (16, 16, 5, 22), (80, 20, 70, 23), (7, 5, 3, 24)]:
        m = wl.random_model(K, 3, 1, W, H, seed=seed, sig_hi=14.0)
        b = oracle.bin(m, 3, 1, W, H)
        ntx, nty = (W + 15) // 16, (H + 15) // 16
        keys, vals, rng = [], [], []
        for t in range(ntx * nty):
            tx, ty = t % ntx, t // ntx
            start = len(keys)
            for j in range(K):
                r = b["tile_rects"][j]
                if r[0] <= tx <= r[2] and r[1] <= ty <= r[3]:
                    keys.append(t)
                    vals.append(j)
            rng.append((start, len(keys)))
        assert b["P"] == len(keys) == int(b["counts"].sum())
        assert np.array_equal(b["keys"], keys) and np.array_equal(b["vals"], vals)
        assert np.array_equal(b["ranges"], np.array(rng).reshape(-1, 2))
        pairs = sorted(zip(keys, vals))
        assert pairs == list(zip(b["keys"].tolist(), b["vals"].tolist()))


# --------------------------------------------------------------------------- gates


def test_untruncated_gates_are_softmax():
    """Untruncated gates w_j = softmax_j(rho_j - q_j/2) (Eq. 4 with pi = e^rho), checked
    with scipy.special.softmax: one-hot constant experts over C = K channels make
    y_c = w_c."""
    from scipy.special import softmax

    W, H, K = 20, 14, 7
    m1 = wl.random_model(K, 1, 0, W, H, seed=31, margin=0.0)
    m = np.zeros((K, 6 + K))
    m[:, :6] = m1[:, :6]
    m[:, 6:] = np.eye(K)
    y, D = oracle.render(m, K, 0, W, H, truncated=False)
    u, v, x, yy = centres(W, H)
    q = maha_np(m1, x, yy)
    ref = softmax(m1[:, 5:6].astype(np.float64) - 0.5 * q, axis=0).T.reshape(H, W, K)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(y.sum(-1), 1.0, rtol=1e-14)


def test_two_kernel_logistic_edge():
    """Two round kernels with equal sigma and pi: w_1 = logistic((q_2 - q_1)/2), exactly
    1/2 on the bisector (the 2D version of the step edge of Fig. 2)."""
    s = 3.0
    m = np.array([[10.5, 8.0, s, 0.0, s, 0.2, 1.0], [16.5, 8.0, s, 0.0, s, 0.2, 0.0]])
    W, H = 27, 16
    y, _ = oracle.render(m, 1, 0, W, H, truncated=False)
    u, v, x, yy = centres(W, H)
    q1 = ((x - 10.5) ** 2 + (yy - 8.0) ** 2) / s ** 2
    q2 = ((x - 16.5) ** 2 + (yy - 8.0) ** 2) / s ** 2
    ref = 1.0 / (1.0 + np.exp(-(q2 - q1) / 2.0))
    np.testing.assert_allclose(y[..., 0].ravel(), ref, rtol=1e-13)
    assert np.all(y[:, 13, 0] == 0.5)  # centre x = 13.5 is the bisector


# --------------------------------------------------------------------------- sharpening


def test_sharpen_steepens_the_logistic_edge_by_f_squared():
    """Native sharpening (Sec. II-B, Fig. 2b): with the bandwidth divided by f, q scales by
    f^2, so the two-kernel edge is logistic(f^2 (q2 - q1) / 2) in the unsharpened q; the
    bisector stays at exactly 1/2 and the flat sides move towards their expert values."""
    s = 3.0
    m = np.array([[10.5, 8.0, s, 0.0, s, 0.2, 1.0], [16.5, 8.0, s, 0.0, s, 0.2, 0.0]])
    W, H = 27, 16
    u, v, x, yy = centres(W, H)
    q1 = ((x - 10.5) ** 2 + (yy - 8.0) ** 2) / s ** 2
    q2 = ((x - 16.5) ** 2 + (yy - 8.0) ** 2) / s ** 2
    prev = None
    for f in (1.0, 1.5, 2.0, 3.0):  # s / f exact in binary32
        ms = oracle.sharpen(m, f)
        assert np.array_equal(ms[:, [0, 1, 5, 6]], m[:, [0, 1, 5, 6]])
        y, _ = oracle.render(ms, 1, 0, W, H, truncated=False)
        ref = 1.0 / (1.0 + np.exp(-f * f * (q2 - q1) / 2.0))
        np.testing.assert_allclose(y[..., 0].ravel(), ref, rtol=1e-12)
        assert np.all(y[:, 13, 0] == 0.5)
        row = y[8, :, 0]
        assert np.all(np.diff(row) <= 0)  # monotone across the edge
        if prev is not None:
            assert row[14] - row[12] < prev[14] - prev[12]  # steeper
            assert np.all(row[:13] >= prev[:13]) and np.all(row[14:] <= prev[14:])
        prev = row


def test_sharpen_by_two_equals_coordinate_scaling_bitwise():
    """Sigma / f^2 at x is Sigma at f x with centres f mu and slopes W / f: the model sharpened
    by 2 rendered at scale 2 equals, bit for bit, the model with doubled centres and halved
    slopes at scale 1 (powers of two scale every binary32 and fp64 step exactly), truncation
    decisions included -- with the ellipse test deciding (the 16x16 native blocks are not
    scaled with the coordinates, so the block lists alone are not)."""
    W, H = 30, 22
    m = wl.random_model(40, 3, 1, W, H, seed=31, sig_lo=0.7, sig_hi=6.0).astype(np.float64)
    m2 = m.copy()
    m2[:, 0:2] *= 2.0
    m2[:, 9:15] *= 0.5
    ms = oracle.sharpen(m, 2.0)
    np.testing.assert_array_equal(ms[:, 2:5] * 2.0, m[:, 2:5])
    ya, Da = oracle.render(ms, 3, 1, 2 * W, 2 * H, s=2, trunc="render")
    yb, Db = oracle.render(m2, 3, 1, 2 * W, 2 * H, s=1, trunc="render")
    np.testing.assert_array_equal(ya, yb)
    np.testing.assert_array_equal(Da, Db)
    assert (Da > 0).sum() > 1000


def test_sharpen_one_or_zero_is_identity():
    m = wl.random_model(10, 3, 1, 20, 20, seed=32).astype(np.float64)
    for f in (0.0, 1.0):
        np.testing.assert_array_equal(oracle.sharpen(m, f), m)


# --------------------------------------------------------------------------- tight box


def aniso_model(K, W, H, seed):
    return wl.stretched_model(K, 3, 1, W, H, seed).astype(np.float64)


def test_tight_box_is_the_ellipse_extent():
    """Half-widths r sqrt(Sigma_xx), r sqrt(Sigma_yy) (Sigma from numpy's L L^T), capped at
    the square box: the oracle's block rectangles equal those of the exact extents wherever
    a block edge does not fall inside the rounding margin."""
    W, H = 70, 54
    compared = 0
    for s, ox, oy in [(1, 0, 0), (2, 3, 5), (3, 1, 0)]:
        m = aniso_model(80, W, H, seed=40 + s)
        S = sigma_of(m)
        lam = np.linalg.eigvalsh(S)[:, 1]
        tr = oracle.bin(m, 3, 1, s * W - ox, s * H - oy, s, ox, oy, box=1)["tile_rects"]
        for j in range(m.shape[0]):
            rng = []
            for k, (mu, o, n) in enumerate([(m[j, 0], ox, s * W - ox), (m[j, 1], oy, s * H - oy)]):
                e = min(R * np.sqrt(S[j, k, k]), R * np.sqrt(lam[j]))
                tight = _np_output_blocks(_np_native_blocks(mu - e, mu + e), n, s, o)
                e2 = min(e * (1 + 2e-3) + 1e-3, R * np.sqrt(lam[j]))
                loose = _np_output_blocks(_np_native_blocks(mu - e2, mu + e2), n, s, o)
                rng.append((tight and tight[0]) if tight == loose else "skip")
            if "skip" in rng:
                continue
            compared += 1
            if rng[0] is None or rng[1] is None:
                assert tr[j, 2] < tr[j, 0], j
            else:
                assert tuple(tr[j]) == (rng[0][0], rng[1][0], rng[0][1], rng[1][1]), (s, j)
    assert compared > 200


def test_tight_box_keeps_every_value_and_shortens_lists():
    """With the ellipse test in the render, the tight box changes no value (the test never
    accepts a pixel outside it) and
    every list is a subset of the square box's list; brute force: every block holding a pixel
    strictly inside the FP64 ellipse is in the kernel's tight rectangle."""
    W, H = 61, 47
    for s, ox, oy, f in [(1, 0, 0, 1.0), (2, 5, 2, 1.0), (3, 0, 7, 1.0), (1, 0, 0, 1.8)]:
        m = oracle.sharpen(aniso_model(90, W, H, seed=50 + s), f)
        OW, OH = s * W - ox, s * H - oy
        ya, Da = oracle.render(m, 3, 1, OW, OH, s, ox, oy, box=0, trunc="render")
        yb, Db = oracle.render(m, 3, 1, OW, OH, s, ox, oy, box=1, trunc="render")
        np.testing.assert_array_equal(ya, yb)
        np.testing.assert_array_equal(Da, Db)
        sq = oracle.bin(m, 3, 1, OW, OH, s, ox, oy, box=0, trunc="render")
        ti = oracle.bin(m, 3, 1, OW, OH, s, ox, oy, box=1, trunc="render")
        assert ti["P"] < 0.8 * sq["P"]
        a, b = sq["tile_rects"], ti["tile_rects"]
        ne = b[:, 2] >= b[:, 0]
        assert np.all(a[ne, 0] <= b[ne, 0]) and np.all(a[ne, 1] <= b[ne, 1])
        assert np.all(a[ne, 2] >= b[ne, 2]) and np.all(a[ne, 3] >= b[ne, 3])
        v, u = np.mgrid[0:OH, 0:OW]
        x, y = (ox + u.ravel() + 0.5) / s, (oy + v.ravel() + 0.5) / s
        q = maha_np(m, x, y)
        for j in range(m.shape[0]):
            hit = q[j] <= R * R * (1 - 1e-6)
            if not hit.any():
                continue
            bx = (ox + u.ravel()[hit]) // 16 - ox // 16
            by = (oy + v.ravel()[hit]) // 16 - oy // 16
            assert b[j, 0] <= bx.min() and bx.max() <= b[j, 2], (s, j)
            assert b[j, 1] <= by.min() and by.max() <= b[j, 3], (s, j)


def test_tight_box_keeps_loss_and_gradient():
    """With the ellipse test in the render, the oracle's loss and gradient sum over pixels and
    participating kernels only, so the tight box gives them bit for bit (one thread: the row-to-thread split of a threaded run,
    and with it the FP64 rounding, varies from run to run)."""
    W, H = 40, 33
    m = aniso_model(50, W, H, seed=58)
    t = np.random.default_rng(2).uniform(0, 1, (H, W, 3))
    la, ga = oracle.loss_grad(m, 3, 1, W, H, target=t, box=0, threads=1, trunc="render")
    lb, gb = oracle.loss_grad(m, 3, 1, W, H, target=t, box=1, threads=1, trunc="render")
    assert la == lb
    np.testing.assert_array_equal(ga, gb)


def test_tight_box_of_round_kernels_is_the_square_box():
    m = wl.random_model(50, 3, 1, 40, 40, seed=60).astype(np.float64)
    m[:, 3] = 0.0
    m[:, 4] = m[:, 2]
    a = oracle.bin(m, 3, 1, 40, 40, box=0)
    b = oracle.bin(m, 3, 1, 40, 40, box=1)
    np.testing.assert_array_equal(a["tile_rects"], b["tile_rects"])


# --------------------------------------------------------------------------- invariants


def test_gates_sum_to_one_all_ones_experts():
    W, H = 45, 38
    m = wl.random_model(50, 3, 1, W, H, seed=41)
    m[:, 6:9] = 1.0
    m[:, 9:] = 0.0
    for trunc in ("render", "gradient"):
        y, D = oracle.render(m, 3, 1, W, H, trunc=trunc)
        cov = D > 0
        assert cov.any() and (trunc == "gradient" or (~cov).any())
        np.testing.assert_allclose(y[cov], 1.0, rtol=1e-14)
        assert np.all(y[~cov] == 0.0)


def test_single_kernel_reproduces_linear_expert():
    """K = 1: the gate is 1 on the kernel's support, so y = a + W (x - mu) there (linear,
    steered expert), with wx multiplying the column offset and wy the row offset."""
    W, H = 40, 33
    m = np.array([[17.3, 15.8, 5.0, 1.5, 3.0, -0.4, 0.2, 0.5, 0.9, 0.011, -0.02, 0.004,
                   -0.013, 0.007, 0.03]])
    y, D = oracle.render(m, 3, 1, W, H)
    u, v, x, yy = centres(W, H)
    on = D.ravel() > 0
    ref = m[0, 6:9] + np.outer(x - m[0, 0], m[0, 9:12]) + np.outer(yy - m[0, 1], m[0, 12:15])
    np.testing.assert_allclose(y.reshape(-1, 3)[on], ref[on], rtol=1e-13, atol=1e-15)
    assert on.sum() > 100


def test_equal_constant_experts_render_the_constant():
    W, H = 31, 29
    m = wl.random_model(40, 1, 0, W, H, seed=42)
    m[:, 6] = 0.3125
    y, D = oracle.render(m, 1, 0, W, H)
    np.testing.assert_allclose(y[D > 0], 0.3125, rtol=1e-14)


def test_integer_translation_equivariance():
    """mu on a 2^-8 grid, integer shift t: render(mu + t)[p + t] = render(mu)[p] -- any shift
    with the ellipse test in the render; shifts by whole blocks with the block lists alone
    deciding the render (the rule then depends on the 16 x 16 grid)."""
    W, H = 64, 48
    m = wl.random_model(30, 3, 1, W, H, seed=43, margin=-8.0).astype(np.float64)
    m[:, :2] = np.round(m[:, :2] * 256) / 256
    for trunc, (tx, ty) in (("render", (5, 3)), ("gradient", (16, 32))):
        y0, D0 = oracle.render(m, 3, 1, W, H, trunc=trunc)
        m2 = m.copy()
        m2[:, 0] += tx
        m2[:, 1] += ty
        y1, D1 = oracle.render(m2, 3, 1, W + tx, H + ty, trunc=trunc)
        np.testing.assert_allclose(y1[ty:, tx:], y0, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(D1[ty:, tx:], D0, rtol=1e-12, atol=1e-300)


def test_subpixel_sampling_scale3():
    """Super-resolution (Sec. II-B, VII-C) re-samples the one regression, under both readings:
    at s = 3 output pixel 3i+1 samples native i + 0.5 (up to the rounding of 1/3), the point
    of native pixel i; an origin shift by any whole number of output pixels is a crop, bit
    for bit."""
    W, H = 30, 26
    m = wl.random_model(25, 3, 1, W, H, seed=44)
    for trunc in ("render", "gradient"):
        y1, _ = oracle.render(m, 3, 1, W, H, trunc=trunc)
        y3, _ = oracle.render(m, 3, 1, 3 * W, 3 * H, s=3, trunc=trunc)
        np.testing.assert_allclose(y3[1::3, 1::3], y1, atol=1e-5)
        yc, _ = oracle.render(m, 3, 1, 40, 35, s=3, ox=11, oy=7, trunc=trunc)
        np.testing.assert_array_equal(yc, y3[7:42, 11:51])
        y1c, _ = oracle.render(m, 3, 1, 19, 13, ox=5, oy=9, trunc=trunc)
        np.testing.assert_array_equal(y1c, y1[9:22, 5:24])


def test_render_is_a_function_of_the_native_point():
    """Whatever raster a point is sampled on (scale 1-4, any origin, ragged sizes), its value
    is the model's value at that native point: every raster's render equals, bit for bit, the
    oracle's evaluation at the raster's binary32 sample points with boxes on the native block
    grid alone -- and the block lists (not only the ellipse) then depend on the point."""
    m = wl.random_model(50, 3, 1, 40, 36, seed=47, sig_lo=0.6, sig_hi=9.0)
    for trunc in ("render", "gradient"):
        for (s, ox, oy, W, H) in [(1, 0, 0, 40, 36), (1, 7, 3, 29, 22), (2, 5, 11, 61, 47),
                                  (3, 13, 2, 77, 59), (4, 9, 30, 83, 71)]:
            y, D = oracle.render(m, 3, 1, W, H, s=s, ox=ox, oy=oy, trunc=trunc)
            pts = oracle.sample_points(W, H, s, ox, oy)
            yp, Dp = oracle.render_points(m, 3, 1, pts.reshape(-1, 2), trunc=trunc)
            np.testing.assert_array_equal(y.reshape(-1, 3), yp)
            np.testing.assert_array_equal(D.ravel(), Dp)


def test_render_points_block_membership_bruteforce():
    """The native block rule at arbitrary points, by brute force in numpy: kernel j takes
    part at x iff floor(x / 16) lies in the native blocks of its box (eigvalsh half-side),
    per axis -- with no cut ("lists"), D is exactly the sum of pi K over those kernels."""
    m = wl.random_model(40, 1, 0, 48, 40, seed=48, sig_lo=0.8, sig_hi=7.0).astype(np.float64)
    rng = np.random.default_rng(49)
    pts = rng.uniform(-8, 56, size=(600, 2)).astype(np.float32)
    _, D = oracle.render_points(m, 1, 0, pts, truncated="lists")
    lam = np.linalg.eigvalsh(sigma_of(m))[:, 1]
    Rj = R * np.sqrt(lam)
    x, y = pts[:, 0].astype(np.float64), pts[:, 1].astype(np.float64)
    q = maha_np(m, x, y)
    ref = np.zeros(pts.shape[0])
    for j in range(m.shape[0]):
        bx = _np_native_blocks(m[j, 0] - Rj[j], m[j, 0] + Rj[j])
        by = _np_native_blocks(m[j, 1] - Rj[j], m[j, 1] + Rj[j])
        if bx is None or by is None:
            continue
        inb = ((np.floor(x / 16) >= bx[0]) & (np.floor(x / 16) <= bx[1]) &
               (np.floor(y / 16) >= by[0]) & (np.floor(y / 16) <= by[1]))
        ref += np.where(inb, np.exp(m[j, 5] - 0.5 * q[j]), 0.0)
    np.testing.assert_allclose(D, ref, rtol=1e-12, atol=1e-300)
    assert (D > 0).sum() > 400


def test_common_pi_scale_invariance():
    W, H = 33, 27
    m = wl.random_model(30, 3, 1, W, H, seed=45).astype(np.float64)
    y0, _ = oracle.render(m, 3, 1, W, H)
    m[:, 5] += 1.75
    y1, _ = oracle.render(m, 3, 1, W, H)
    np.testing.assert_allclose(y1, y0, rtol=1e-12, atol=1e-14)


def test_sampled_pixels_equal_full_raster():
    W, H = 37, 21
    m = wl.random_model(20, 3, 1, W, H, seed=46)
    y, D = oracle.render(m, 3, 1, W, H)
    pix = [(0, 0), (36, 20), (17, 3), (5, 19)]
    ys, Ds = oracle.render(m, 3, 1, W, H, pixels=pix)
    for i, (u, v) in enumerate(pix):
        assert np.array_equal(ys[i], y[v, u]) and Ds[i] == D[v, u]


# --------------------------------------------------------------------------- gradients


def _fd_guard(model, W, H, margin=1e-4):
    u, v, x, y = centres(W, H)
    q = maha_np(model, x, y)
    assert np.min(np.abs(q - R * R)) > margin, "a (pixel, kernel) pair sits on the truncation edge"


def test_gradient_central_differences():
    """Analytic gradient of the MSE (raw parameters, Cholesky log-diagonal) against FP64
    central differences, h = 1e-6, on a 32x32 crop with K = 16 linear experts -- with the
    ellipse test in the render, where the gradient is the rendered loss's."""
    tgt, raw = wl.fd_crop_case()
    H, W, C = tgt.shape
    raw = raw.astype(np.float64)
    model = oracle.materialize(raw, 3, 1)
    _fd_guard(model, W, H)
    loss, g = oracle.loss_grad(model, 3, 1, W, H, target=tgt, trunc="render")
    h = 1e-6
    fd = np.zeros_like(g)
    for j in range(raw.shape[0]):
        for k in range(raw.shape[1]):
            rp = raw.copy(); rp[j, k] += h
            rm = raw.copy(); rm[j, k] -= h
            lp, _ = oracle.loss_grad(oracle.materialize(rp, 3, 1), 3, 1, W, H, target=tgt,
                                    trunc="render")
            lm, _ = oracle.loss_grad(oracle.materialize(rm, 3, 1), 3, 1, W, H, target=tgt,
                                    trunc="render")
            fd[j, k] = (lp - lm) / (2 * h)
    groups = {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5], "a": [6, 7, 8],
              "wx": [9, 10, 11], "wy": [12, 13, 14]}
    for name, cols in groups.items():
        ref = fd[:, cols]
        err = np.max(np.abs(g[:, cols] - ref)) / np.max(np.abs(ref))
        assert err < 2e-5, (name, err)
        assert np.max(np.abs(ref)) > 0


def test_gradient_rho_sums_to_zero():
    """Gates sum to one at every covered pixel, so a common shift of all rho changes
    nothing: sum_j dL/drho_j = 0."""
    tgt, raw = wl.fd_crop_case(seed=7)
    H, W, _ = tgt.shape
    model = oracle.materialize(raw.astype(np.float64), 3, 1)
    _, g = oracle.loss_grad(model, 3, 1, W, H, target=tgt, trunc="render")
    assert abs(g[:, 5].sum()) < 1e-12 * np.abs(g[:, 5]).sum()
    assert np.abs(g[:, 5]).max() > 1e-6


def test_gradient_constant_expert_sum_closed_form():
    """Constant experts: sum_j dL/da_jc = sum over covered pixels of dL/dy_c = 2 (y_c - t_c)/N."""
    img = wl.config1_image()
    raw, model = wl.grid_init(img, 8, 8, 4.0, order=0)
    model = model.astype(np.float64)
    rng = np.random.default_rng(5)
    model[:, :2] += rng.uniform(-2, 2, size=(64, 2))
    model[:, 6] += rng.uniform(-0.1, 0.1, size=64)
    H, W, _ = img.shape
    y, D = oracle.render(model, 1, 0, W, H, trunc="render")
    loss, g = oracle.loss_grad(model, 1, 0, W, H, target=img, trunc="render")
    gy = 2 * (y - img) / (H * W)
    assert g[:, 6].sum() == pytest.approx(gy[D > 0].sum(), rel=1e-11)
    assert loss == pytest.approx(np.mean((y - img) ** 2), rel=1e-13)


def test_upstream_gradient_mode_and_subsets():
    """grad_y mode with dL/dy = 2(y - t)/N equals the fused-MSE gradient, and requesting a
    subset of kernels returns the same rows."""
    tgt, raw = wl.fd_crop_case(seed=9)
    H, W, _ = tgt.shape
    model = oracle.materialize(raw.astype(np.float64), 3, 1)
    _, g = oracle.loss_grad(model, 3, 1, W, H, target=tgt)
    y, _ = oracle.render(model, 3, 1, W, H)
    _, g2 = oracle.loss_grad(model, 3, 1, W, H, grad_y=2 * (y - tgt) / y.size)
    np.testing.assert_allclose(g2, g, rtol=1e-12, atol=1e-18)
    sel = [3, 0, 11]
    _, g3 = oracle.loss_grad(model, 3, 1, W, H, target=tgt, kernels=sel)
    np.testing.assert_allclose(g3, g[sel], rtol=1e-12, atol=1e-18)


# --------------------------------------------------------------------------- optimizer


def test_adam_matches_torch_optim_adam():
    """Adam with per-group learning rates and the exponential centre-rate decay, against
    torch.optim.Adam in float64 fed the same gradients."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    K, C, order = 9, 3, 1
    NP = 15
    p = rng.normal(size=(K, NP))
    grads = [rng.normal(size=(K, NP)) * 10.0 ** rng.uniform(-4, 0) for _ in range(6)]
    lr = dict(mu=1e-2, mu_final=1e-5, chol=1e-3, rho=2e-3, expert=5e-3)
    total = 6
    tp = torch.tensor(p.copy(), dtype=torch.float64)
    cols = {"mu": [0, 1], "chol": [2, 3, 4], "rho": [5], "expert": list(range(6, NP))}
    params = {k: tp[:, c].clone().requires_grad_(True) for k, c in cols.items()}
    opt = torch.optim.Adam([{"params": [params[k]], "lr": lr[k]} for k in cols],
                           betas=(0.9, 0.999), eps=1e-8)
    pp, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for t, g in enumerate(grads):
        lrs = oracle.step_lrs(t, total, lr["mu"], lr["mu_final"], lr["chol"], lr["rho"], lr["expert"])
        oracle.adam(pp, g, m, v, t + 1, lrs, C, order)
        opt.param_groups[0]["lr"] = lr["mu"] * (lr["mu_final"] / lr["mu"]) ** (t / total)
        for k, c in cols.items():
            params[k].grad = torch.tensor(g[:, c], dtype=torch.float64)
        opt.step()
    out = np.zeros_like(p)
    for k, c in cols.items():
        out[:, c] = params[k].detach().numpy()
    np.testing.assert_allclose(pp, out, rtol=1e-12, atol=1e-14)


def test_fit_one_step_equals_materialize_grad_adam():
    """oracle_fit is materialize -> loss/gradient -> Adam; one step reproduces the pieces."""
    img = wl.config1_image()
    raw, _ = wl.grid_init(img, 8, 8, 4.0, order=0)
    raw = raw.astype(np.float64)
    hist, out = oracle.fit(raw, 1, 0, img, steps=1, lr_mu=1e-2, lr_chol=1e-2, lr_rho=1e-2,
                           lr_expert=1e-2)
    model = oracle.materialize(raw, 1, 0)
    loss, g = oracle.loss_grad(model, 1, 0, 64, 64, target=img)
    p, m, v = raw.copy(), np.zeros_like(raw), np.zeros_like(raw)
    oracle.adam(p, g, m, v, 1, [1e-2] * 4, 1, 0)
    assert hist[0] == pytest.approx(loss, rel=1e-14)
    np.testing.assert_allclose(out, p, rtol=1e-14, atol=1e-15)


def test_fit_reduces_loss_workload1():
    """100 Adam steps on the 64x64 grey workload lower the MSE (trajectory itself is
    parity-unpinned: FP32 and FP64 runs legitimately diverge)."""
    w = wl.workload(1)
    hist, out = oracle.fit(w.raw0, 1, 0, w.target, steps=100, lr_mu=1e-2, lr_chol=1e-2,
                           lr_rho=1e-2, lr_expert=1e-2)
    assert hist[-1] < 0.7 * hist[0]
    assert np.all(np.isfinite(out))


# --------------------------------------------------------------------------- RBF sum (Eq. 1)


def test_rbf_single_kernel_closed_form():
    """Eq. (1) with one kernel, untruncated: y_c = pi K(x) m_c(x), K from numpy's Mahalanobis
    form, m the linear expert; D = pi K as in the gated mode."""
    W, H = 21, 17
    m = wl.random_model(5, 3, 1, W, H, seed=70, margin=0.0).astype(np.float64)
    u, v, x, y = centres(W, H)
    q = maha_np(m, x, y)
    for j in range(m.shape[0]):
        yr, D = oracle.render(m[j:j + 1], 3, 1, W, H, truncated=False, rbf=True)
        e = np.exp(m[j, 5] - 0.5 * q[j])
        dx, dy = x - m[j, 0], y - m[j, 1]
        for c in range(3):
            ref = e * (m[j, 6 + c] + m[j, 9 + c] * dx + m[j, 12 + c] * dy)
            np.testing.assert_allclose(yr[..., c].ravel(), ref, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(D.ravel(), e, rtol=1e-12)


def test_rbf_superposition_and_numerator():
    """Eq. (1) is additive over kernels (a model's render is the sum of its halves' renders,
    truncated or not) and equals the gated mode's numerator y_smoe D."""
    W, H = 45, 38
    m = wl.random_model(80, 3, 1, W, H, seed=71, sig_lo=0.7, sig_hi=8.0).astype(np.float64)
    for trunc in (True, False):
        y, _ = oracle.render(m, 3, 1, W, H, truncated=trunc, rbf=True)
        ya, _ = oracle.render(m[:37], 3, 1, W, H, truncated=trunc, rbf=True)
        yb, _ = oracle.render(m[37:], 3, 1, W, H, truncated=trunc, rbf=True)
        np.testing.assert_allclose(y, ya + yb, rtol=1e-12, atol=1e-14)
        ys, Ds = oracle.render(m, 3, 1, W, H, truncated=trunc)
        np.testing.assert_allclose(y, ys * Ds[..., None], rtol=1e-12, atol=1e-14)


def test_rbf_gradient_central_differences():
    """Analytic gradient of the MSE of the RBF sum against FP64 central differences (h = 1e-6)
    on the 32x32 crop with K = 16 linear experts."""
    tgt, raw = wl.fd_crop_case(seed=11)
    H, W, C = tgt.shape
    raw = raw.astype(np.float64)
    model = oracle.materialize(raw, 3, 1)
    _fd_guard(model, W, H)
    _, g = oracle.loss_grad(model, 3, 1, W, H, target=tgt, rbf=True, trunc="render")
    h = 1e-6
    fd = np.zeros_like(g)
    for j in range(raw.shape[0]):
        for k in range(raw.shape[1]):
            rp = raw.copy(); rp[j, k] += h
            rm = raw.copy(); rm[j, k] -= h
            lp, _ = oracle.loss_grad(oracle.materialize(rp, 3, 1), 3, 1, W, H, target=tgt, rbf=True,
                                    trunc="render")
            lm, _ = oracle.loss_grad(oracle.materialize(rm, 3, 1), 3, 1, W, H, target=tgt, rbf=True,
                                    trunc="render")
            fd[j, k] = (lp - lm) / (2 * h)
    groups = {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5], "a": [6, 7, 8],
              "wx": [9, 10, 11], "wy": [12, 13, 14]}
    for name, cols in groups.items():
        ref = fd[:, cols]
        err = np.max(np.abs(g[:, cols] - ref)) / np.max(np.abs(ref))
        assert err < 2e-5, (name, err)
        assert np.max(np.abs(ref)) > 0


def test_rbf_rho_gradient_closed_form():
    """Constant experts in Eq. (1): y = sum_j pi_j a_j K_j, so dL/drho_j = sum_c a_jc dL/da_jc
    (pi and a enter as a product); the gated mode has no such identity."""
    W, H = 40, 36
    m = wl.random_model(60, 3, 0, W, H, seed=72, sig_lo=1.0, sig_hi=6.0).astype(np.float64)
    t = np.random.default_rng(4).uniform(0, 1, (H, W, 3))
    _, g = oracle.loss_grad(m, 3, 0, W, H, target=t, rbf=True)
    ref = (m[:, 6:9] * g[:, 6:9]).sum(axis=1)
    np.testing.assert_allclose(g[:, 5], ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())
    _, gs = oracle.loss_grad(m, 3, 0, W, H, target=t)
    assert not np.allclose(gs[:, 5], (m[:, 6:9] * gs[:, 6:9]).sum(axis=1), rtol=1e-3)


# --------------------------------------------------------------- ellipse in the gradient only


def _np_block_rects(m, W, H):
    """Square-box block rectangles of the native raster in FP64 numpy: half-side
    r sqrt(lambda_max) from eigvalsh of L L^T, the native pixel centres in the box, their
    blocks, clamped to the raster's."""
    lam = np.linalg.eigvalsh(sigma_of(m))[:, 1]
    Rj = R * np.sqrt(lam)
    out = []
    for j in range(m.shape[0]):
        bx = _np_output_blocks(_np_native_blocks(m[j, 0] - Rj[j], m[j, 0] + Rj[j]), W)
        by = _np_output_blocks(_np_native_blocks(m[j, 1] - Rj[j], m[j, 1] + Rj[j]), H)
        out.append(None if bx is None or by is None else (bx[0][0], by[0][0], bx[0][1], by[0][1]))
    return out


# A listed term is rendered iff binary32 holds it: rho log2(e) - q log2(e)/2 >= -125.
ARG_MIN = -125.0


def _np_arg(m, q):
    return m[:, 5:6] * math.log2(math.e) - 0.5 * math.log2(math.e) * q


def _np_blocklist_terms(m, C, order, W, H, rects):
    """Per (kernel, pixel): whether the kernel takes part in the render (its block list holds
    the pixel's block and binary32 holds its term), pi K, q, and the experts' values
    [K, n, C] (numpy FP64, native raster)."""
    u, v, x, y = centres(W, H)
    q = maha_np(m, x, y)
    arg = _np_arg(m, q)
    cover = np.zeros(q.shape, dtype=bool)
    for j, rc in enumerate(rects):
        if rc is not None:
            cover[j] = ((u >> 4) >= rc[0]) & ((u >> 4) <= rc[2]) & ((v >> 4) >= rc[1]) & \
                       ((v >> 4) <= rc[3]) & (arg[j] >= ARG_MIN)
    e = np.where(cover, np.exp(m[:, 5:6] - 0.5 * q), 0.0)
    dx, dy = x[None, :] - m[:, 0:1], y[None, :] - m[:, 1:2]
    ex = np.stack([m[:, 6 + c:7 + c] + (m[:, 6 + C + c:7 + C + c] * dx +
                                        m[:, 6 + 2 * C + c:7 + 2 * C + c] * dy if order else 0.0)
                   for c in range(C)], axis=-1)
    return cover, e, q, ex


def _np_blocklist_render(m, C, order, W, H, rects):
    _, e, _, ex = _np_blocklist_terms(m, C, order, W, H, rects)
    D = e.sum(axis=0)
    N = (e[..., None] * ex).sum(axis=0)
    y = np.where(D[:, None] > 0, N / np.where(D > 0, D, 1.0)[:, None], 0.0)
    return y.reshape(H, W, C), D.reshape(H, W)


def test_blocklist_render_bruteforce():
    """Sec. IV-B with the discard in the gradient only: every kernel of a block's list takes
    part at every pixel of the block whose term binary32 holds.  numpy FP64 brute force
    (boxes from eigvalsh, Gaussians from numpy.linalg.solve) against the oracle's render."""
    for (W, H, K, seed) in [(45, 38, 40, 81), (32, 32, 8, 82), (70, 20, 60, 83)]:
        m = wl.random_model(K, 3, 1, W, H, seed=seed, sig_lo=0.7, sig_hi=9.0).astype(np.float64)
        rects = _np_block_rects(m, W, H)
        tr = oracle.bin(m, 3, 1, W, H)["tile_rects"]
        for j, rc in enumerate(rects):
            assert (tuple(tr[j]) == rc) if rc is not None else tr[j, 2] < tr[j, 0], j
        cover, _, q, _ = _np_blocklist_terms(m, 3, 1, W, H, rects)
        # pixels with a pair at the render's edge are left out (binary32 forms the exponent
        # within ~1e-4 of FP64 there, so either side may keep the term)
        near = (np.abs(_np_arg(m, q) - ARG_MIN) < 2e-3).any(axis=0).reshape(H, W)
        assert near.sum() <= 3
        y_np, D_np = _np_blocklist_render(m, 3, 1, W, H, rects)
        y, D = oracle.render(m, 3, 1, W, H)
        np.testing.assert_allclose(D[~near], D_np[~near], rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(y[~near], y_np[~near], rtol=1e-11, atol=1e-13)
        # some pixels take kernels beyond their ellipse, which the other reading drops
        y_r, _ = oracle.render(m, 3, 1, W, H, trunc="render")
        assert np.max(np.abs(y - y_r)) > 1e-6


def test_gradient_only_ellipse_per_pair_differences():
    """The gradient with out-of-ellipse pixels discarded (Sec. IV-B): kernel j's gradient is
    the sum, over the pixels inside its ellipse, of the derivative of that pixel's squared
    error with respect to j's raw parameters (render over the block lists, rule held fixed).
    Brute force: FP64 central differences of every pixel's error, h = 1e-6, masked by numpy's
    q <= r^2, on a 32x32 RGB case with 6 linear experts."""
    W = H = 32
    C, order = 3, 1
    m0 = wl.random_model(6, C, order, W, H, seed=84, sig_lo=2.0, sig_hi=7.0, margin=0.0)
    m0 = m0.astype(np.float64)
    raw = m0.copy()
    raw[:, 2], raw[:, 4] = np.log(m0[:, 2]), np.log(m0[:, 4])
    tgt = np.random.default_rng(85).uniform(0, 1, (H, W, C))
    rects = _np_block_rects(m0, W, H)
    cover, _, q, _ = _np_blocklist_terms(m0, C, order, W, H, rects)
    assert np.min(np.abs(q - R * R)) > 1e-4
    assert np.min(np.abs(_np_arg(m0, q) - ARG_MIN)) > 2e-3
    inside = cover & (q <= R * R)
    assert (cover & ~inside).any()

    def pixel_errors(r):
        mm = r.copy()
        mm[:, 2], mm[:, 4] = np.exp(r[:, 2]), np.exp(r[:, 4])
        y, _ = _np_blocklist_render(mm, C, order, W, H, rects)
        return ((y - tgt) ** 2).sum(axis=-1).ravel() / (W * H * C)

    h = 1e-6
    fd = np.zeros_like(raw)
    for j in range(raw.shape[0]):
        for k in range(raw.shape[1]):
            rp = raw.copy(); rp[j, k] += h
            rm = raw.copy(); rm[j, k] -= h
            fd[j, k] = ((pixel_errors(rp) - pixel_errors(rm)) / (2 * h))[inside[j]].sum()
    _, g = oracle.loss_grad(m0, C, order, W, H, target=tgt)
    groups = {"mu": [0, 1], "s1": [2], "l21": [3], "s2": [4], "rho": [5], "a": [6, 7, 8],
              "wx": [9, 10, 11], "wy": [12, 13, 14]}
    for name, cols in groups.items():
        ref = fd[:, cols]
        err = np.max(np.abs(g[:, cols] - ref)) / np.max(np.abs(ref))
        assert err < 2e-5, (name, err)
    # and it is not the rendered loss's full gradient
    full = np.zeros_like(raw)
    for j in range(raw.shape[0]):
        rp = raw.copy(); rp[j, 6] += h
        rm = raw.copy(); rm[j, 6] -= h
        full[j, 6] = ((pixel_errors(rp) - pixel_errors(rm)) / (2 * h))[cover[j]].sum()
    assert np.max(np.abs(full[:, 6] - g[:, 6])) > 1e-3 * np.max(np.abs(g[:, 6]))


# --------------------------------------------------------------------------- golden


def _golden(name):
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k1, v1, k2, v2 = line.split()
                rows[(k1, float(v1))] = (k2, float(v2))
    return rows


def test_confidence_ellipse_mass_golden():
    """Sec. IV-B's 99 % confidence ellipse: the fixture's radius and mass, checked by the
    closed form and by integrating the oracle's untruncated single-kernel render over a fine
    raster (the fraction of its mass inside q <= r^2, which the render-side ellipse test
    keeps)."""
    g = _golden("confidence_ellipse.txt")
    r99 = g[("mass", 0.99)][1]
    m3 = g[("radius", 3.0)][1]
    assert r99 == pytest.approx(math.sqrt(-2 * math.log(0.01)), rel=1e-15)
    assert m3 == pytest.approx(1 - math.exp(-4.5), rel=1e-15)
    # one round kernel, sigma = 4 native px, on a raster reaching 6 sigma from its centre,
    # sampled at scale 4 (pixel area 1/16)
    s, sig, W = 4, 4.0, 192
    m = np.array([[W / (2 * s), W / (2 * s), sig, 0.0, sig, 0.0, 1.0]])
    _, D_all = oracle.render(m, 1, 0, W, W, s=s, truncated=False)
    for r, mass in ((3.0, m3), (r99, 0.99)):
        _, D_in = oracle.render(m, 1, 0, W, W, s=s, r=r, trunc="render")
        assert D_in.sum() / D_all.sum() == pytest.approx(mass, abs=2e-3)


# ---------------------------------------------------------------- the render's cut, measured


def test_render_cut_loses_nothing_against_the_uncut_block_lists():
    """Eq. (5) over the block lists has no cut; binary32 cannot hold a term below its normal
    range, so the render keeps exactly the listed terms with exponent >= -125.  On a model
    the oracle fitted (the 64x64 workload, 100 Adam steps) and on stretched models with
    mixing weights spread over rho in [-3, 3], the default render equals the uncut FP64
    block-list sum and leaves no pixel uncovered; a cut at q <= (2r)^2 would change y by
    more than 1e-6 on the stretched models (numpy FP64 brute force)."""
    w = wl.workload(1)
    _, raw = oracle.fit(w.raw0, 1, 0, w.target, 100, lr_mu=1e-2, lr_chol=1e-2, lr_rho=1e-2,
                        lr_expert=1e-2)
    cases = [(oracle.materialize(raw, 1, 0), 1, 0, 64, 64)]
    for seed in (1, 2):
        ms = wl.stretched_model(300, 3, 1, 96, 80, seed).astype(np.float64)
        ms[:, 5] = np.random.default_rng(seed).uniform(-3, 3, ms.shape[0])
        cases.append((ms, 3, 1, 96, 80))
    worst_2r = 0.0
    for m, C, order, W, H in cases:
        y, D = oracle.render(m, C, order, W, H)
        yu, Du = oracle.render(m, C, order, W, H, truncated="lists")
        assert np.max(np.abs(y - yu)) <= 1e-14
        assert (D == 0).sum() == 0 and (Du == 0).sum() == 0
        rects = _np_block_rects(m, W, H)
        u, v, x, yy = centres(W, H)
        q = maha_np(m, x, yy)
        cover = np.zeros(q.shape, dtype=bool)
        for j, rc in enumerate(rects):
            if rc is not None:
                cover[j] = ((u >> 4) >= rc[0]) & ((u >> 4) <= rc[2]) & ((v >> 4) >= rc[1]) & \
                           ((v >> 4) <= rc[3]) & (q[j] <= 4 * R * R)
        e = np.where(cover, np.exp(m[:, 5:6] - 0.5 * q), 0.0)
        dx, dy = x[None, :] - m[:, 0:1], yy[None, :] - m[:, 1:2]
        ex = np.stack([m[:, 6 + c:7 + c] + (m[:, 6 + C + c:7 + C + c] * dx +
                                            m[:, 6 + 2 * C + c:7 + 2 * C + c] * dy if order else 0.0)
                       for c in range(C)], axis=-1)
        Dc = e.sum(axis=0)
        yc = ((e[..., None] * ex).sum(axis=0) / Dc[:, None]).reshape(H, W, C)
        worst_2r = max(worst_2r, float(np.max(np.abs(yc - yu))))
    assert worst_2r > 1e-6


def test_output_blocks_never_straddle_native_blocks():
    """Output blocks are aligned to multiples of 16 in o + u, so that at every integer scale a
    native block (16 s output pixels) begins on an output block boundary: the sample point of
    output coordinate G = o + u, fl(fl(G + 1/2) fl(1/s)) in binary32, lies in native block
    floor(G / (16 s)).  Exhaustively, for every scale the ABI accepts (1-64) and every native
    boundary G = 16 k s over the accepted coordinate range (|o| <= 2^22, widths <= 65536): the
    points on both sides of each boundary fall in the blocks on their sides.  The GPU renders
    a block's list without a per-point membership test on the strength of this."""
    lo, hi = -(1 << 22), (1 << 22) + 65536
    for s in range(1, 65):
        inv = np.float32(1.0) / np.float32(s)
        k = np.arange(lo // (16 * s) - 1, hi // (16 * s) + 2, dtype=np.int64)
        for g, want in ((16 * k * s - 1, k - 1), (16 * k * s, k)):
            m = (g >= lo) & (g < hi)
            x = (g[m].astype(np.float32) + np.float32(0.5)) * inv
            nb = np.floor(x * np.float32(0.0625)).astype(np.int64)
            assert np.array_equal(nb, want[m]), s
