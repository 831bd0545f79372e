"""Mutation check of the oracle's pins.

Each case plants one plausible mistake (a dropped term, a wrong sign, index or
base, a transposed operand) into a temporary copy of ``oracle/rs_oracle.c``,
builds it with gcc on the CPU and runs the pins of ``test_oracle_pins`` against
the mutant.  Every mutant must fail at least one pin; the real oracle (built
by the session fixture) passes them all in ``test_oracle_pins``.
"""
import os
import tempfile

import pytest

import oracle
import tests.test_oracle_pins as pins

MUTATIONS = {
    "natural_log": ("H -= p * log2(p);", "H -= p * log(p);"),
    "drop_L_factor": ("return H * (double)L;", "return H;"),
    "keep_v_equals_u": ("if (v == u || w == u || v == w)", "if (w == u || v == w)"),
    "no_cw_ne_cv": ("if (lab[w] == lab[u] || lab[w] == lab[v])", "if (lab[w] == lab[u])"),
    "drop_open_type2": ("return closed ? 3 : 2;", "return closed ? 3 : 0;"),
    "drop_closed_type2": ("return closed ? 3 : 2;", "return closed ? 0 : 2;"),
    "count_open_type1": ("return closed ? 1 : 0;", "return 1;"),
    "denominator_d_squared": ("double dd = (double)(d * (d - 1));", "double dd = (double)(d * d);"),
    "transposed_weight": ("rso_triad_term(lookup(&o, v, lab[u]), lookup(&o, w, lab[v]),",
                          "rso_triad_term(lookup(&o, v, lab[u]), lookup(&o, v, lab[w]),"),
    "wrong_reference": ("lookup(&o, w, lab[u]));", "lookup(&o, w, lab[w]));"),
    "omega_max_without_own": ("        if (o->w_own[v] > m)\n            m = o->w_own[v];\n", ""),
    "no_omega_max_division": ("sum_norm += t / omax;", "sum_norm += t;"),
    "reference_in_Y": ("        if (comms[i] == ref)\n            continue;\n        Y += (double)counts[i];",
                       "        Y += (double)counts[i];\n        if (comms[i] == ref)\n            continue;"),
    "square_root": ("return cbrt(w_vu * w_wv * w_wu);", "return sqrt(w_vu * w_wv * w_wu);"),
    "tie_break_reversed": ("    return (x > y) - (x < y);\n}\n\n/* K highest", "    return (x < y) - (x > y);\n}\n\n/* K highest"),
    "accept_self_loop": ("if (v < 0 || v >= n || v == u)", "if (v < 0 || v >= n)"),
}

PIN_TESTS = [
    pins.test_worked_example_weight,
    pins.test_worked_example_normalization,
    pins.test_worked_example_rsi,
    pins.test_k4_four_communities_closed_form,
    pins.test_entropy_two_to_one,
    pins.test_at_most_two_labels_scores_zero,
    pins.test_single_foreign_community_neighbourhood,
    pins.test_degree_one_and_isolated,
    pins.test_brute_force_agrees,
    pins.test_bfs_robustness_of_counted_triads,
    pins.test_topk_ties_and_bounds,
]


def _fails_some_pin(lib):
    for t in PIN_TESTS:
        try:
            t(lib)
        except (AssertionError, RuntimeError):
            return True
    for case in ("self",):
        try:
            pins.test_validate_rejects(case, lib)
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(name):
    src = open(oracle.SRC).read()
    old, new = MUTATIONS[name]
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mut.c")
        so = os.path.join(d, "mut.so")
        open(c, "w").write(mutated)
        import subprocess
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                        "-o", so, c, "-lm"], check=True)
        lib = oracle.load(so)
        assert _fails_some_pin(lib), f"no pin catches mutation {name}"
