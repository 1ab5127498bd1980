"""Planted mistakes: each plausible slip in the oracle must fail at least one pin.

Every case copies oracle/hough_oracle.c, changes one expression (a sign, an
operand, a dropped term, an edge test, the tie rule, the wrap, the sort key),
builds the copy with the oracle's own flags, and runs the pins of
test_oracle_pins.py against it in a child process.  Nothing here touches the
GPU or the HIP library.
"""

import json
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

MUTANTS = {
    "num_sign_of_d0": ("float num = 2.0f * (u - d);", "float num = 2.0f * (u + d);"),
    "den_cross_term_sign": ("float den = r2 - 2.0f * d * u + d * d;", "float den = r2 + 2.0f * d * u + d * d;"),
    "den_dropped_d0_squared": ("float den = r2 - 2.0f * d * u + d * d;", "float den = r2 - 2.0f * d * u;"),
    "u_transposed_operands": ("float u = yi * c - xi * s;", "float u = xi * c - yi * s;"),
    "u_sign": ("float u = yi * c - xi * s;", "float u = xi * s - yi * c;"),
    "r2_wrong_term": ("float r2 = xi * xi + yi * yi;", "float r2 = xi * xi + xi * yi;"),
    "d0_ignored": ("float d = d0 ? d0[l] : 0.0f;", "float d = 0.0f;"),
    "kappa_offset_sign": ("float kf = (kappa - kappa_min) * kappa_scale;",
                          "float kf = (kappa + kappa_min) * kappa_scale;"),
    "lower_edge_exclusive": ("if (kf >= 0.0f && kf < n_kappa_f)", "if (kf > 0.0f && kf < n_kappa_f)"),
    "threshold_strict": ("if (v < threshold)", "if (v <= threshold)"),
    "tie_rule_kappa_axis": ("int negative = od != 0 ? od < 0 : (op != 0 ? op < 0 : ok < 0);",
                            "int negative = od != 0 ? od < 0 : (op != 0 ? op < 0 : ok > 0);"),
    "tie_rule_all_strict": ("if (negative ? !(v > w) : !(v >= w))", "if (!(v > w))"),
    "phi_not_periodic": ("                if (jj < 0)\n                    jj += n_phi;\n"
                         "                if (jj >= n_phi)\n                    jj -= n_phi;\n",
                         "                if (jj < 0 || jj >= n_phi)\n                    continue;\n"),
    "sort_votes_ascending": ("return a->votes > b->votes ? -1 : 1;", "return a->votes < b->votes ? -1 : 1;"),
    "sort_cells_descending": ("return a->cell < b->cell ? -1 : 1;", "return a->cell > b->cell ? -1 : 1;"),
    "vertex_column_num_sign": ("float num = dt + t;", "float num = dt - t;"),
    "vertex_row_num_sign": ("float num = t - dt;", "float num = t + dt;"),
    "vertex_d0_ignored": ("const float dt = d0 ? d0[l] : 0.0f;", "const float dt = 0.0f;"),
    "vertex_mode_inverted": ("if (fabsf(c) >= fabsf(s)) {", "if (fabsf(c) < fabsf(s)) {"),
    "vertex_column_uses_cos": ("float t = x_centre[ix] * s;", "float t = x_centre[ix] * c;"),
    "vertex_row_divides_by_cos": ("float xv = num / s;", "float xv = num / c;"),
    "vertex_y_offset_sign": ("float fy = (yv - y_min) * y_scale;", "float fy = (yv + y_min) * y_scale;"),
    "vertex_y_lower_edge_exclusive": ("if (fy >= 0.0f && fy < n_y_f)", "if (fy > 0.0f && fy < n_y_f)"),
    "vertex_x_lower_edge_exclusive": ("if (fx >= 0.0f && fx < n_x_f)", "if (fx > 0.0f && fx < n_x_f)"),
    "vertex_phi_row_decoding": ("const int32_t j = (int32_t)((cell / n_kappa) % n_phi);",
                                "const int32_t j = (int32_t)(cell % n_phi);"),
    "vertex_track_threshold_strict": ("if (cand_votes[i] < track_threshold)", "if (cand_votes[i] <= track_threshold)"),
    "vertex_tie_rule_y_axis": ("const int negative = dx != 0 ? dx < 0 : dy < 0;",
                               "const int negative = dx != 0 ? dx < 0 : dy > 0;"),
    "vertex_peaks_x_periodic": ("const int32_t xx = ix + dx;", "const int32_t xx = (ix + dx + n_x) % n_x;"),
    "vertex_peak_threshold_strict": ("if (val < threshold)", "if (val <= threshold)"),
    "straight_u_sign": ("float along = yh * cos_phi[j] - xh * sin_phi[j];",
                        "float along = yh * cos_phi[j] + xh * sin_phi[j];"),
    "straight_u_transposed": ("float along = yh * cos_phi[j] - xh * sin_phi[j];",
                              "float along = xh * cos_phi[j] - yh * sin_phi[j];"),
    "straight_offset_sign": ("float fd = (along - d0_min) * d0_scale;", "float fd = (along + d0_min) * d0_scale;"),
    "straight_lower_edge_exclusive": ("if (fd >= 0.0f && fd < n_d0_f)", "if (fd > 0.0f && fd < n_d0_f)"),
    "forward_not_strict": ("if (!(ahead > 0.0f))", "if (!(ahead >= 0.0f))"),
    "forward_term_sign": ("float ahead = xi * c + yi * s;", "float ahead = xi * c - yi * s;"),
    "forward_uses_the_offset": ("float ahead = xi * c + yi * s;", "float ahead = yi * c - xi * s;"),
    "forward_backward": ("if (!(ahead > 0.0f))", "if (!(ahead < 0.0f))"),
    "straight_forward_backward": ("if (!(fwd > 0.0f))", "if (!(fwd < 0.0f))"),
    "straight_forward_operands": ("float fwd = xh * cos_phi[j] + yh * sin_phi[j];",
                                  "float fwd = yh * cos_phi[j] + xh * sin_phi[j];"),
    "assoc_kappa_window_one_sided": ("k >= kc - 1 && k <= kc + 1", "k >= kc && k <= kc + 1"),
    "assoc_phi_not_periodic": ("const int32_t jj = (jc + dj + n_phi) % n_phi;",
                               "const int32_t jj = jc + dj < 0 || jc + dj >= n_phi ? jc : jc + dj;"),
    "assoc_d0_window_dropped": ("for (int dl = -1; dl <= 1 && !member; ++dl) {",
                                "for (int dl = 0; dl <= 0 && !member; ++dl) {"),
    "assoc_forward_ignored": ("        if (!(front > 0.0f))\n            return 0;\n", ""),
    "assoc_straight_uses_curvature": ("if (family == 1) {", "if (family == 2) {"),
    "assoc_chord_sign": ("float chord2 = hr2 - 2.0f * dl0 * off + dl0 * dl0;",
                         "float chord2 = hr2 + 2.0f * dl0 * off + dl0 * dl0;"),
}

RUNNER = r"""
import json, sys, inspect
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, test_oracle_pins as P
P.LIBRARY[0] = oracle.load_library({lib!r})
with open(P.GOLDEN) as f:
    golden = json.load(f)
cases = []
for name, fn in sorted(vars(P).items()):
    if not name.startswith("test_"):
        continue
    marks = getattr(fn, "pytestmark", [])
    params = [m for m in marks if m.name == "parametrize"]
    if params:
        argnames = [a.strip() for a in params[0].args[0].split(",")]
        for vals in params[0].args[1]:
            vals = vals if len(argnames) > 1 else (vals,)
            cases.append((name + str(vals), fn, dict(zip(argnames, vals))))
    elif "golden" in inspect.signature(fn).parameters:
        cases.append((name, fn, {{"golden": golden}}))
    else:
        cases.append((name, fn, {{}}))
failed = []
for name, fn, kw in cases:
    try:
        fn(**kw)
    except Exception as e:
        failed.append(name)
print(json.dumps({{"failed": failed, "n": len(cases)}}))
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(src.replace(old, new))
    lib = oracle.build(str(mutant_src), str(tmp_path / "libmutant.so"))
    code = RUNNER.format(root=os.path.dirname(HERE), tests=HERE, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["n"] > 10
    assert out["failed"], f"no pin caught the planted mistake {name}"


def test_unmutated_oracle_passes_every_pin(tmp_path):
    lib = oracle.build(oracle.SRC, str(tmp_path / "libclean.so"))
    code = RUNNER.format(root=os.path.dirname(HERE), tests=HERE, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["failed"] == []
