"""Planted mistakes in a copy of the oracle must fail at least one pin.

Each mutant is a plausible slip (a swapped tap, a dropped term, a wrong
sign, focal length or comparison) applied textually to oracle/bn_oracle.c,
compiled to a temporary library and run through every check in pins.py.
This shows the pins constrain each part of the oracle, not just some.
"""
import os
import subprocess

import pytest

import oracle
import pins
import pins_variants

MUTANTS = {
    "eq10_fx_for_fy": [("n[0] = -alpha / (4.0 * fy)", "n[0] = -alpha / (4.0 * fx)")],
    "eq12_drop_alpha2_term": [("+ alpha * alpha / (4.0 * fx * fy) * (d2 + d4) * (d3 + d5);", "+ 0.0;")],
    "eq12_sign_u1": [("n[2] = -u1 * n[0] - v1 * n[1]", "n[2] = u1 * n[0] - v1 * n[1]")],
    "u1_with_fy": [("double u1 = ((double)x - cx) / fx;", "double u1 = ((double)x - cx) / fy;")],
    "taps_3_5_swapped": [("(y + alpha) * stride + x]", "(y + ALPHA_MINUS) * stride + x]"),
                         ("(y - alpha) * stride + x]", "(y + alpha) * stride + x]"),
                         ("(y + ALPHA_MINUS) * stride + x]", "(y - alpha) * stride + x]")],
    "eq7_wrong_pair": [("cross3(s15, s12, c)", "cross3(s12, s15, c)")],
    "not_camera_facing": [("out[0] = -n[0] / len;", "out[0] = n[0] / len;"),
                          ("out[1] = -n[1] / len;", "out[1] = n[1] / len;"),
                          ("out[2] = -n[2] / len;", "out[2] = n[2] / len;")],
    "border_off_by_one": [("(x - alpha >= 0)", "(x - alpha >= -1)")],
    "d1_not_checked": [("tap_ok_f32(d1) && ", "")],
    "mask_not_strict": [("(q > h) ?", "(q >= h) ?")],
    "rel_tau_not_squared": [("float tt = tau * tau;", "float tt = tau;")],
    "abs_threshold_not_squared": [("    k = k * k;\n", "")],
    "xc_uses_cy": [("float xc = (float)x - cx;", "float xc = (float)x - cy;")],
    "my_uses_fx": [("float my = fy * b;", "float my = fx * b;")],
    "no_degenerate_rule": [("if (!isfinite(q) || q < FLT_MIN)", "if (!isfinite(q))")],
    "boundary_keeps_normal": [("if (code == ORC_VALID) {", "if (code != ORC_INVALID) {")],
    "q_missing_mz": [("float q = (mx2 + my2) + mz2;", "float q = (mx2 + my2);")],
    # row bands: output indexed by the full-frame row instead of the band row
    "band_rows_full_frame_index": [("int64_t i = (int64_t)(y - row_begin) * W + x;",
                                    "int64_t i = (int64_t)y * W + x;")],
    # pair removal
    "pair_34_wrong_direction": [("const int sh[4] = {1, -1, -1, 1};",
                                 "const int sh[4] = {1, 1, -1, 1};")],
    "pair_taps_regrouped": [("const int tv[4] = {3, 3, 5, 5};", "const int tv[4] = {3, 5, 3, 5};")],
    "pair_keep_inverted": [("if (!fire) k |= 1 << p;", "if (fire) k |= 1 << p;")],
    "pair_average_ignores_test": [("        if (!(keep & (1 << p)))\n            continue;\n"
                                   "        n[0] += np[p][0];", "        n[0] += np[p][0];")],
    "pair_abs_without_alpha": [("    k = k / (double)alpha;\n    k = k * k;\n    return (float)k;\n}\n\n"
                                "static float multiscale_abs",
                                "    k = k * k;\n    return (float)k;\n}\n\nstatic float multiscale_abs")],
    "pair_definition_wrong_order": [("static const int PAIR_K[4] = {3, 4, 5, 2};",
                                     "static const int PAIR_K[4] = {3, 2, 5, 4};")],
    # the fused binary32 pair sequence (methods 1 and 2)
    "pair_mz_offsets_swapped": [("float z = fmaf(xc, A, fmaf(yc, B, w));",
                                 "float z = fmaf(xc, B, fmaf(yc, A, w));")],
    "pair_q_missing_my": [("*q = fmaf(x, x, fmaf(y, y, z * z));", "*q = fmaf(x, x, z * z);")],
    "pair_w_wrong_tap": [("w[p] = (af * d[th[p]]) * d[tv[p]];", "w[p] = (af * d[th[p]]) * d[th[p]];")],
    "pair_rel_threshold_not_squared": [("float h = tw * w[p];", "float h = tw;")],
    "pair_sum_q_missing_z": [("float Q = fmaf(sx, sx, fmaf(sy, sy, sz * sz));",
                              "float Q = fmaf(sx, sx, sy * sy);")],
    "pair_closed_form_mz_sign": [("float cz = fmaf(xc, a, fmaf(yc, b, cw));",
                                  "float cz = fmaf(xc, a, fmaf(yc, b, -cw));")],
    "ms_q_missing_mz": [("float q = fmaf(Mx, Mx, fmaf(My, My, Mz * Mz));",
                         "float q = fmaf(Mx, Mx, My * My);")],
    # multi-scale
    "ms_same_offset_every_scale": [("float a = (float)(i * alpha);", "float a = (float)alpha;")],
    "ms_unweighted_scales": [("Mx = a * mx;", "Mx = mx;"), ("My = a * my;", "My = my;"),
                             ("Mz = a * mz;", "Mz = mz;"), ("Wt = a * w;", "Wt = w;"),
                             ("Mx = fmaf(a, mx, Mx);", "Mx = Mx + mx;"),
                             ("My = fmaf(a, my, My);", "My = My + my;"),
                             ("Mz = fmaf(a, mz, Mz);", "Mz = Mz + mz;"),
                             ("Wt = fmaf(a, w, Wt);", "Wt = Wt + w;")],
    "ms_abs_without_K": [("    double k = (double)scales;\n    k = k * (double)fx;",
                          "    double k = 1.0;\n    k = k * (double)fx;")],
    "ms_border_both_sides": [("int inside = (x + reach <= W - 1) && (y + reach <= H - 1);",
                              "int inside = (x + reach <= W - 1) && (y + reach <= H - 1) && "
                              "(x - reach >= 0);")],
    "ms_sum_not_averaged": [("    n[0] /= scales;\n    n[1] /= scales;\n    n[2] /= scales;\n", "")],
    "ms_eq2_fx_for_fy": [("n[1] = -a / fx * d2 * (d3 - d1);", "n[1] = -a / fy * d2 * (d3 - d1);")],
    "ms_eq3_sign_u1": [("+ a / fy * u1 * d3 * (d2 - d1)", "- a / fy * u1 * d3 * (d2 - d1)")],
}


def _apply(src, edits):
    for old, new in edits:
        assert old in src, f"mutation anchor not found: {old!r}"
        src = src.replace(old, new)
    return src


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oracle.SRC).read()
    mutated = _apply(src, MUTANTS[name])
    assert mutated != src
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, str(c), "-o", str(so), "-lm"])
    o = oracle.Oracle(str(so))
    failed = []
    for pin in pins.ALL_PINS + pins_variants.VARIANT_PINS:
        try:
            pin(o)
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
