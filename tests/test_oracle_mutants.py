"""Planted mistakes: each plausible slip in the oracle must fail at least one pin.

Every case copies oracle/hough_oracle.c, changes one expression (a sign, an
operand, a dropped term, an edge test, the tie rule, the wrap, the sort key,
or the binary32 operation order: a reassociation, a fused multiply-add, a
division through a reciprocal, a distributed product, binary64 evaluation),
builds the copy with the oracle's own flags, and runs the pins of
test_oracle_pins.py against it in a child process.  One more case builds the
unchanged source with contraction allowed (-ffp-contract=fast -mfma).  Exact
rewrites -- forms that round identically for every input the vote can see --
must pass every pin, so the pins check the arithmetic and not its spelling.
Nothing here touches the GPU or the HIP library.
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
    # the binary32 operation order of the vote (caught by tests/golden/fp32_order.json)
    "r2_contracted_x": ("float r2 = xi * xi + yi * yi;", "float r2 = fmaf(xi, xi, yi * yi);"),
    "r2_contracted_y": ("float r2 = xi * xi + yi * yi;", "float r2 = fmaf(yi, yi, xi * xi);"),
    "u_contracted_yc": ("float u = yi * c - xi * s;", "float u = fmaf(yi, c, -(xi * s));"),
    "u_contracted_xs": ("float u = yi * c - xi * s;", "float u = fmaf(-xi, s, yi * c);"),
    "den_reassociated": ("float den = r2 - 2.0f * d * u + d * d;", "float den = r2 + (d * d - 2.0f * d * u);"),
    "den_square_first": ("float den = r2 - 2.0f * d * u + d * d;", "float den = (r2 + d * d) - 2.0f * d * u;"),
    "den_contracted_cross": ("float den = r2 - 2.0f * d * u + d * d;",
                             "float den = fmaf(-2.0f * d, u, r2) + d * d;"),
    "den_contracted_square": ("float den = r2 - 2.0f * d * u + d * d;",
                              "float den = fmaf(d, d, r2 - 2.0f * d * u);"),
    "kappa_by_reciprocal": ("float kappa = num / den;", "float kappa = num * (1.0f / den);"),
    "kf_distributed": ("float kf = (kappa - kappa_min) * kappa_scale;",
                       "float kf = kappa * kappa_scale - kappa_min * kappa_scale;"),
    "kf_contracted": ("float kf = (kappa - kappa_min) * kappa_scale;",
                      "float kf = fmaf(kappa, kappa_scale, -(kappa_min * kappa_scale));"),
    "vote_in_double": ("                float u = yi * c - xi * s;\n"
                       "                float num = 2.0f * (u - d);\n"
                       "                float den = r2 - 2.0f * d * u + d * d;\n"
                       "                float kappa = num / den;\n"
                       "                float kf = (kappa - kappa_min) * kappa_scale;\n",
                       "                double u = (double)yi * c - (double)xi * s;\n"
                       "                double num = 2.0 * (u - d);\n"
                       "                double den = ((double)xi * xi + (double)yi * yi) - 2.0 * d * u + (double)d * d;\n"
                       "                double kappa = num / den;\n"
                       "                double kf = (kappa - kappa_min) * (double)kappa_scale;\n"),
    "straight_u_contracted": ("float along = yh * cos_phi[j] - xh * sin_phi[j];",
                              "float along = fmaf(yh, cos_phi[j], -(xh * sin_phi[j]));"),
    "straight_fd_distributed": ("float fd = (along - d0_min) * d0_scale;",
                                "float fd = along * d0_scale - d0_min * d0_scale;"),
    "straight_fd_contracted": ("float fd = (along - d0_min) * d0_scale;",
                               "float fd = fmaf(along, d0_scale, -(d0_min * d0_scale));"),
    "vertex_column_contracted": ("float num = dt + t;", "float num = fmaf(x_centre[ix], s, dt);"),
    "vertex_column_reciprocal": ("float yv = num / c;", "float yv = num * (1.0f / c);"),
    "vertex_fy_distributed": ("float fy = (yv - y_min) * y_scale;", "float fy = yv * y_scale - y_min * y_scale;"),
    "vertex_row_contracted": ("float num = t - dt;", "float num = fmaf(y_centre[iy], c, -dt);"),
    "vertex_row_reciprocal": ("float xv = num / s;", "float xv = num * (1.0f / s);"),
    "vertex_fx_distributed": ("float fx = (xv - x_min) * x_scale;", "float fx = xv * x_scale - x_min * x_scale;"),
    "assoc_r2_contracted": ("const float hr2 = hx * hx + hy * hy;", "const float hr2 = fmaf(hx, hx, hy * hy);"),
    "assoc_off_contracted": ("float off = hy * cj - hx * sj;", "float off = fmaf(hy, cj, -(hx * sj));"),
    "assoc_chord_reassociated": ("float chord2 = hr2 - 2.0f * dl0 * off + dl0 * dl0;",
                                 "float chord2 = hr2 + (dl0 * dl0 - 2.0f * dl0 * off);"),
    "assoc_curv_reciprocal": ("float curv = twice / chord2;", "float curv = twice * (1.0f / chord2);"),
    "assoc_frac_distributed": ("frac = (curv - kmin) * kscale;", "frac = curv * kscale - kmin * kscale;"),
    "assoc_straight_frac_distributed": ("frac = (off - kmin) * kscale;", "frac = off * kscale - kmin * kscale;"),
}

# Rewrites that round exactly as the canonical order for every input the vote
# can see (finite, no overflow): 2*(u - d) = 2u - 2d because doubling is exact;
# (2d)*u = 2*(d*u) for the same reason; in 2D (d = +0, den = r2) the quotient
# 2u/r2 is the real number u/(r2/2), and halving r2 is exact, so the correctly
# rounded quotients agree.  The device uses the last form.
EXACT_REWRITES = {
    "num_distributed": ("float num = 2.0f * (u - d);", "float num = 2.0f * u - 2.0f * d;"),
    "den_cross_term_regrouped": ("float den = r2 - 2.0f * d * u + d * d;",
                                 "float den = r2 - 2.0f * (d * u) + d * d;"),
    "kappa_over_half_r2_in_2d": ("float kappa = num / den;",
                                 "float kappa = d0 == NULL ? u / (0.5f * r2) : num / den;"),
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


def _cpu_has_fma():
    try:
        with open("/proc/cpuinfo") as f:
            return any(line.startswith("flags") and " fma " in line + " " for line in f)
    except OSError:
        return False


@pytest.mark.skipif(not _cpu_has_fma(), reason="the host CPU has no fused multiply-add")
def test_contracted_build_fails_a_pin(tmp_path):
    """The unchanged source built with contraction allowed: the compiler fuses
    products into sums wherever it likes, which the order fixture must see."""
    lib = oracle.build(oracle.SRC, str(tmp_path / "libcontracted.so"), extra=["-ffp-contract=fast", "-mfma"])
    code = RUNNER.format(root=os.path.dirname(HERE), tests=HERE, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["failed"], "no pin caught the contracted build"


@pytest.mark.parametrize("name", sorted(EXACT_REWRITES))
def test_exact_rewrite_passes_every_pin(name, tmp_path):
    old, new = EXACT_REWRITES[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"rewrite anchor for {name} not found exactly once"
    rewrite_src = tmp_path / "rewrite.c"
    rewrite_src.write_text(src.replace(old, new))
    lib = oracle.build(str(rewrite_src), str(tmp_path / "librewrite.so"))
    code = RUNNER.format(root=os.path.dirname(HERE), tests=HERE, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["failed"] == [], f"the exact rewrite {name} failed {out['failed']}"


def test_unmutated_oracle_passes_every_pin(tmp_path):
    lib = oracle.build(oracle.SRC, str(tmp_path / "libclean.so"))
    code = RUNNER.format(root=os.path.dirname(HERE), tests=HERE, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["failed"] == []
