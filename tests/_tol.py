"""Tolerances shared by the GPU parity tests.

The denominator D = sum pi K of a pixel is a sum of binary32 terms 2^a with
a = fma(q, -log2(e)/2, rho log2(e)).  q carries a relative rounding error of a few ulps
(four rounded operations) and a one more, so a term's relative error grows with its exponent:
|dD / D| <= ln(2) |da| + (exp2's ulp) with |da| <~ 5 |a| 2^-24 and |a| ~ |ln D| / ln 2.
Pixels whose D is made of far terms (q up to ~170 when the block lists decide the render)
therefore carry relative errors above 1e-5 in D alone -- the image y = N / D does not, since N
and D share the terms.  The D bar is 1e-5 relative plus 6 |ln D| 2^-24."""
import numpy as np

D_RTOL = 1e-5


def d_rel_error(D, D_ref):
    """max |D - D_ref| / (D_ref (1 + 6 |ln D_ref| 2^-24 / D_RTOL)), to be compared with
    D_RTOL (pixels with D_ref = 0 must have D = 0)."""
    D = np.asarray(D, dtype=np.float64)
    D_ref = np.asarray(D_ref, dtype=np.float64)
    on = D_ref > 0
    assert np.array_equal(D > 0, on)
    if not on.any():
        return 0.0
    scale = 1.0 + 6.0 * np.abs(np.log(D_ref[on])) * 2.0 ** -24 / D_RTOL
    return float(np.max(np.abs(D[on] - D_ref[on]) / (D_ref[on] * scale)))
