"""Planted mistakes: each plausible slip in the oracle must fail at least one pin.

Every case copies the oracle source, applies one textual change (a dropped term, a
flipped sign, swapped axes, a wrong index or normalisation), builds the copy into a
temporary library, re-binds the oracle module to it and runs the pins named for that
case.  The test passes when at least one of those pins fails.  Everything happens on
the CPU; the real oracle library is rebound afterwards.
"""
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = oracle._SRC.read_text()

# (label, original text, planted text, pins expected to catch it)
MUTANTS = [
    ("drop rho in the gate", "t.e = std::exp(r[5] - 0.5 * q);", "t.e = std::exp(-0.5 * q);",
     [pins.test_denominator_is_pi_times_gaussian_eq2_eq4]),
    ("sign of l21 in forward substitution", "t.z2 = (t.dy - r[3] * t.z1) / r[4];",
     "t.z2 = (t.dy + r[3] * t.z1) / r[4];", [pins.test_denominator_is_pi_times_gaussian_eq2_eq4]),
    ("l11 and l22 swapped", "t.z1 = t.dx / r[2];", "t.z1 = t.dx / r[4];",
     [pins.test_denominator_is_pi_times_gaussian_eq2_eq4]),
    ("pixel centre not at +0.5", "return ((float)(o + u) + 0.5f) * inv_s;",
     "return ((float)(o + u) + 0.0f) * inv_s;", [pins.test_hand_computed_single_kernel]),
    ("expert slopes transposed",
     "if (order == 1) m += r[6 + C + c] * dx + r[6 + 2 * C + c] * dy;",
     "if (order == 1) m += r[6 + C + c] * dy + r[6 + 2 * C + c] * dx;",
     [pins.test_single_kernel_reproduces_linear_expert]),
    ("box from sxx instead of lambda_max", "const float lam = h + std::sqrt(d * d + sxy * sxy);",
     "const float lam = sxx;", [pins.test_box_half_side_is_r_sqrt_lambda_max]),
    ("ellipse radius off", "return rule == RULE_ELLIPSE ? q <= r2 :",
     "return rule == RULE_ELLIPSE ? q <= 1.1f * r2 :",
     [pins.test_truncation_rule_matches_ellipse_and_stays_in_box]),
    ("native block rect off by one", "*b1 = native_block(b);", "*b1 = native_block(b) + 1.0f;",
     [pins.test_box_half_side_is_r_sqrt_lambda_max]),
    ("overlapped blocks one short under the ellipse reading",
     "*b1 = std::ceil(hi * 0.0625f) - 1.0f;", "*b1 = std::floor(hi * 0.0625f) - 1.0f;",
     [pins.test_tight_box_keeps_every_value_and_shortens_lists]),
    ("native blocks of 8 pixels", "return std::floor(x * 0.0625f);",
     "return std::floor(x * 0.125f);", [pins.test_render_points_block_membership_bruteforce]),
    ("output blocks counted from the window's first pixel",
     "static int block_start(int t, int o) { return 16 * (first_block(o) + t) - o; }",
     "static int block_start(int t, int o) { return 16 * t; }",
     [pins.test_box_half_side_is_r_sqrt_lambda_max]),
    ("membership from the raster's pixel instead of the native point",
     "const float bx = native_block(x32), by = native_block(y32);",
     "const float bx = native_block(x32 - 0.5f), by = native_block(y32 - 0.5f);",
     [pins.test_render_points_block_membership_bruteforce]),
    ("representable exponent bound off", "return arg >= -125.0f;", "return arg >= -25.0f;",
     [pins.test_blocklist_render_bruteforce]),
    ("no normalisation of the gates", "((Dsum > 0.0) ? N[c] / Dsum : 0.0);",
     "((Dsum > 0.0) ? N[c] : 0.0);", [pins.test_untruncated_gates_are_softmax]),
    ("z2 chain term sign in the gradient", "const double bz1 = -Hh * t.z1 - bz2 * r[3] / r[4];",
     "const double bz1 = -Hh * t.z1 + bz2 * r[3] / r[4];", [pins.test_gradient_central_differences]),
    ("expert slope dropped from d/dmu", "const double bdx = bz1 / r[2] + ex;",
     "const double bdx = bz1 / r[2];", [pins.test_gradient_central_differences]),
    ("l21 gradient missing 1/l22", "out[3] += -bz2 * t.z1 / r[4];", "out[3] += -bz2 * t.z1;",
     [pins.test_gradient_central_differences]),
    ("gradient of y_c uses y of another channel",
     "(g.rbf ? 0.0 : y[c]));",
     "(g.rbf ? 0.0 : y[0]));",
     [pins.test_gradient_central_differences]),
    ("loss mean over H*W only", "const double inv_n = 1.0 / ((double)W * H * C);",
     "const double inv_n = 1.0 / ((double)W * H);", [pins.test_upstream_gradient_mode_and_subsets]),
    ("Adam without bias correction", "const double mhat = m[i] / bc1;", "const double mhat = m[i];",
     [pins.test_adam_matches_torch_optim_adam]),
    ("centre-rate decay exponent inverted",
     "f = std::pow(lr_mu_final / lr_mu, (double)step_index / (double)total_steps);",
     "f = std::pow(lr_mu / lr_mu_final, (double)step_index / (double)total_steps);",
     [pins.test_adam_matches_torch_optim_adam]),
    ("tight box y extent from l22 alone",
     "Ry = std::fmin(R, g.r * std::sqrt(syy) * 1.0009765625f + m);",
     "Ry = std::fmin(R, g.r * std::fabs(l22) * 1.0009765625f + m);",
     [pins.test_tight_box_keeps_every_value_and_shortens_lists,
      pins.test_tight_box_is_the_ellipse_extent]),
    ("tight box axes swapped",
     "native_axis(mux - Rx, mux + Rx, centres, &rc.bx0, &rc.bx1)",
     "native_axis(mux - Ry, mux + Ry, centres, &rc.bx0, &rc.bx1)",
     [pins.test_tight_box_keeps_every_value_and_shortens_lists,
      pins.test_tight_box_is_the_ellipse_extent]),
    ("RBF sum still normalised", "y[c] = g.rbf ? N[c] : ((Dsum",
     "y[c] = g.rbf ? N[c] / Dsum : ((Dsum",
     [pins.test_rbf_single_kernel_closed_form, pins.test_rbf_superposition_and_numerator]),
    ("RBF gradient through the gate", "const double w = g.rbf ? t.e : t.e / D;",
     "const double w = t.e / D;", [pins.test_rbf_gradient_central_differences]),
    ("render drops out-of-ellipse pairs under the block-list reading",
     "(g.trunc == 1 ? RULE_LISTS : RULE_ELLIPSE)", "RULE_ELLIPSE",
     [pins.test_blocklist_render_bruteforce]),
    ("gradient keeps out-of-ellipse pairs",
     "if (!M.participates(j, x32, y32, RULE_ELLIPSE, r2)) continue;",
     "if (!M.participates(j, x32, y32, RULE_LISTS, r2)) continue;",
     [pins.test_gradient_only_ellipse_per_pair_differences]),
    ("block list not in kernel order",
     "for (int j = 0; j < K; ++j) {\n    const Rect32& rc = M.rect[j];\n    int32_t* tr",
     "for (int jj = 0; jj < K; ++jj) {\n    const int j = K - 1 - jj;\n    const Rect32& rc = M.rect[j];\n    int32_t* tr",
     [pins.test_bins_bruteforce_tiny]),
]


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    yield tmp_path_factory.mktemp("mutants")
    oracle.use_library(None)


@pytest.mark.parametrize("label,old,new,catchers", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(workdir, label, old, new, catchers):
    assert SRC.count(old) == 1, f"mutation anchor not unique or missing: {label}"
    idx = MUTANTS.index(next(m for m in MUTANTS if m[0] == label))
    src = workdir / f"m{idx}.cpp"
    so = workdir / f"m{idx}.so"
    src.write_text(SRC.replace(old, new))
    subprocess.check_call(["g++", *oracle.CXXFLAGS, str(src), "-o", str(so)])
    oracle.use_library(so)
    try:
        caught = False
        for pin in catchers:
            try:
                pin()
            except AssertionError:
                caught = True
        assert caught, f"planted mistake not detected: {label}"
    finally:
        oracle.use_library(None)
