"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each mutation is a plausible misreading or slip (wrong vertex decreased,
missing rule, wrong tie-break, wrong rounding, ...).  The mutated source is
compiled into a temporary library and the pin suite is run against it in a
subprocess; the suite must fail.  The real oracle source is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "exactz_oracle.cpp")

MUTATIONS = {
    "v2_decreases_g_argmin": ("if (G.desc != R.desc[i]) mark[R.desc[i]] = 1;",
                              "if (G.desc != R.desc[i]) mark[G.desc] = 1;"),
    "v1_decreases_f_argmax": ("if (G.asc != R.asc[i]) mark[G.asc] = 1;",
                              "if (G.asc != R.asc[i]) mark[R.asc[i]] = 1;"),
    "v3_decreases_upper_end": ("if (lower_f != lower_g) mark[lower_f ? p.second : i] = 1;",
                               "if (lower_f != lower_g) mark[lower_f ? i : p.second] = 1;"),
    "no_spurious_saddle_rule": ("(R.type[i] == TYPE_REGULAR && G.type == TYPE_SADDLE)",
                                "false"),
    "v4_decreases_upper_cp": ("if (lt(g, R.cps[k + 1], R.cps[k])) mark[R.cps[k]] = 1;",
                              "if (lt(g, R.cps[k + 1], R.cps[k])) mark[R.cps[k + 1]] = 1;"),
    "tie_break_reversed": ("return h[i] < h[j] || (h[i] == h[j] && i < j);",
                           "return h[i] < h[j] || (h[i] == h[j] && i > j);"),
    "lower_bound_rounded_to_nearest": ("  fesetround(FE_UPWARD);\n  volatile T lo = a - b;",
                                       "  fesetround(FE_TONEAREST);\n  volatile T lo = a - b;"),
    "lossless_one_edit_early": ("if (c > N) {", "if (c >= N) {"),
    "edit_not_clamped": ("v = cand < Lb[t] ? Lb[t] : cand;", "v = cand;"),
    "step_divides_by_n_plus_1": ("const T delta = step_size(xiT, N);",
                                 "const T delta = step_size(xiT, N + 1);"),
    "descent_over_open_neighbourhood": ("  L.desc = i;\n  L.lower = 0;",
                                        "  L.desc = nb.empty() ? i : nb[0].second;\n  L.lower = 0;"),
    # original event constraints (Sec. 4.2)
    "c2_deleted": ("if (lt(g, R.saddles[k + 1], R.saddles[k])) mark[R.saddles[k]] = 1;",
                   "if (false) mark[R.saddles[k]] = 1;"),
    "c2_decreases_upper_saddle": (
        "if (lt(g, R.saddles[k + 1], R.saddles[k])) mark[R.saddles[k]] = 1;",
        "if (lt(g, R.saddles[k + 1], R.saddles[k])) mark[R.saddles[k + 1]] = 1;"),
    "c3_join_deleted": ("      if (R.lc[s] >= 2) {\n        int64_t sel", "      if (false) {\n        int64_t sel"),
    "c3_split_deleted": ("      if (R.uc[s] >= 2) {\n        int64_t sel", "      if (false) {\n        int64_t sel"),
    "c3_join_lowers_f_choice": ("if (sel >= 0 && sel != R.mf[k]) mark[sel] = 1;",
                                "if (sel >= 0 && sel != R.mf[k]) mark[R.mf[k]] = 1;"),
    "c3_split_lowers_g_choice": ("if (sel >= 0 && sel != R.Mf[k]) mark[R.Mf[k]] = 1;",
                                 "if (sel >= 0 && sel != R.Mf[k]) mark[sel] = 1;"),
    "c3_join_lowers_lower_in_f": (
        "if (sel >= 0 && sel != R.mf[k]) mark[sel] = 1;",
        "if (sel >= 0 && sel != R.mf[k]) mark[lt(f, sel, R.mf[k]) ? sel : R.mf[k]] = 1;"),
    "c3_split_lowers_lower_in_f": (
        "if (sel >= 0 && sel != R.Mf[k]) mark[R.Mf[k]] = 1;",
        "if (sel >= 0 && sel != R.Mf[k]) mark[lt(f, sel, R.Mf[k]) ? sel : R.Mf[k]] = 1;"),
    "c3_join_selects_lowest_minimum_in_g": ("if (sel < 0 || lt(g, sel, t)) sel = t;",
                                            "if (sel < 0 || lt(g, t, sel)) sel = t;"),
    "c3_split_selects_highest_maximum_in_g": ("if (sel < 0 || lt(g, t, sel)) sel = t;",
                                              "if (sel < 0 || lt(g, sel, t)) sel = t;"),
    "c3_join_selects_lowest_minimum_in_f": ("if (R.mf[k] < 0 || lt(f, R.mf[k], t)) R.mf[k] = t;",
                                            "if (R.mf[k] < 0 || lt(f, t, R.mf[k])) R.mf[k] = t;"),
    "c3_paths_start_at_f_lower_link": ("if (glower >> p.first & 1u) {",
                                       "if (R.lower[s] >> p.first & 1u) {"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mutated = tmp_path / "mutant.cpp"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-frounding-math",
                           "-fPIC", "-shared", str(mutated), "-o", str(so)])
    env = dict(os.environ, EXACTZ_ORACLE_SO=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "mutation %s survived the pins:\n%s" % (name, r.stdout[-2000:])
