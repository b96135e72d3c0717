"""Plant plausible mistakes in a copy of the oracle source; the pins must catch each one.

Every mutant is a text replacement in a temporary copy of oracle/gempe_oracle.c, built with
the same flags.  A mutant that no pin rejects would mean the pins cannot tell that mistake
from the paper's definitions, so the test fails.
"""
import os

import pytest

import oracle
import pins

MUTANTS = {
    "edge_sign_swapped": ("double a = is_edge ? -1.0 : 1.0;", "double a = is_edge ? 1.0 : -1.0;"),
    "slope_missing_sigma": ("if (d1) *d1 = -(a / sigma) * R / ORACLE_LN2;",
                            "if (d1) *d1 = -a * R / ORACLE_LN2;"),
    "natural_log_bits": ("if (dl) *dl = -log_Phi(tau) / ORACLE_LN2;", "if (dl) *dl = -log_Phi(tau);"),
    "gradient_sign": ("gi[k] += c * (xi[k] - xj[k]);", "gi[k] += c * (xj[k] - xi[k]);"),
    "gradient_not_unit": ("double c = (delta > 0.0) ? d1 / delta : 0.0;", "double c = d1;"),
    "loss_both_triangles": ("if (j > i) {", "if (j != i) {"),
    "membership_wrong_index": ("int edge = flag[j] != 0;", "int edge = flag[i] != 0;"),
    "erfc_missing_sqrt2": ("return log1p(-0.5 * erfc(t / ORACLE_SQRT2));",
                           "return log1p(-0.5 * erfc(t));"),
    "tail_series_sign": ("q * (3.0 + q * (-15.0", "q * (3.0 + q * (15.0"),
    "tail_log_term": ("- log(-t) - ORACLE_LOG_SQRT_2PI", "+ log(-t) - ORACLE_LOG_SQRT_2PI"),
    "second_derivative_sign": ("(tau * R + R * R)", "(tau * R - R * R)"),
    "distance_not_squared": ("r2 += t * t;", "r2 += fabs(t);"),
    "hist_edge_tau_sign": ("if (e > 0) F += e * (-t) * mills_inv(-t);", "if (e > 0) F += e * t * mills_inv(t);"),
    "hist_bin_lower_edge": ("double delta = sqrt((b + 0.5) * r2_max / nbins);",
                            "double delta = sqrt(b * r2_max / nbins);"),
    "hist_edge_row_flag": ("if (flag[j]) he[b] += 1;", "if (flag[i]) he[b] += 1;"),
    "pairs_edge_sign": ("double a = flag[j] ? -1.0 : 1.0;", "double a = flag[j] ? 1.0 : -1.0;"),
    "lcg_increment": ("state = 1103515245u * state + 1u;", "state = 1103515245u * state;"),
    "draw_rounds_to_nearest": ("int c = (int)floorf(u);", "int c = (int)lrintf(u);"),
    "draw_keeps_neighbours": ("if (is_edge(row_ptr, col_idx, v, c)) continue;", ""),
    "sample_side_swapped": ("samples[2 * e + 1] = draw_non_neighbour(j, n, s1,", "samples[2 * e + 1] = draw_non_neighbour(i, n, s1,"),
    "sampled_edge_as_non_edge": ("add_pair(d, X, i, j, 1, mu, sigma, Y, Z, &loss);", "add_pair(d, X, i, j, 0, mu, sigma, Y, Z, &loss);"),
    "bisection_direction": ("if (Fn(s, ctx) < 0.0) lo = s; else hi = s;", "if (Fn(s, ctx) < 0.0) hi = s; else lo = s;"),
    "shard_by_larger_vertex": ("int lo = i < j ? i : j;", "int lo = i < j ? j : i;"),
    "shard_strips_unpaired": ("int p = q < S - 1 - q ? q : S - 1 - q;", "int p = q;"),
    "shard_owner_shifted": ("return p % G == s;", "return (p + 1) % G == s;"),
    "wm_weight_full_curvature": ("                    double w = 0.5 * d2;", "                    double w = d2;"),
    "sampled_weight_full_curvature": ("\n    double w = 0.5 * d2;", "\n    double w = d2;"),
    "abs_slope_scaled": ("A += fabs(d1);", "A += 100.0 * fabs(d1);"),
    "abs_slope_over_distance": ("A += fabs(d1);", "A += fabs(d1) / delta;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, oracle_mod, name):
    src = open(oracle.source_path()).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor not unique for {name}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(path), str(tmp_path / f"libmutant_{name}.so"))
    caught = []
    oracle.use_library(lib)
    try:
        for pin in pins.ALL_PINS:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
                break
    finally:
        oracle.use_library(None)
    assert caught, f"no pin rejects mutant {name}"
