"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a wrong sign or index, a transposed operand, a swapped convention),
builds it on the CPU and runs a subset of the pins from test_oracle_pins.py
against it: at least one pin must fail.  The unmodified source must pass the
same subset.
"""
import os
import subprocess
import sys

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "lbp_oracle.c")

MUTATIONS = {
    "dense_table_first_slot_fastest": (
        "for (int32_t l = arity - 1; l > j; --l)", "for (int32_t l = 0; l < j; ++l)"),
    "explicit_table_column_major": (
        "g->tab_states[g->tab_off[t] + c * arity + j]",
        "g->tab_states[g->tab_off[t] + j * g->tab_ncfg[t] + c]"),
    "damping_weights_swapped": (
        "m_next[o + s] = d * m[o + s] + (1.0 - d) * u[o + s];",
        "m_next[o + s] = (1.0 - d) * m[o + s] + d * u[o + s];"),
    "no_normalisation": (
        "for (int32_t s = 0; s < ns; ++s) m_next[o + s] -= mx;", ""),
    "belief_without_evidence": (
        "double b = g->theta[g->vs_off[v] + s];", "double b = 0.0;"),
    "vtof_without_leave_one_out": (
        "            n[g->es_off[e] + s] = B[g->vs_off[v] + s] - m[g->es_off[e] + s];\n    }\n    int64_t mc",
        "            n[g->es_off[e] + s] = B[g->vs_off[v] + s];\n    }\n    int64_t mc"),
    "enum_missing_self_subtraction": (
        "u[g->es_off[e] + s] = lse_t(sel, cnt, T) - n[g->es_off[e] + s];",
        "u[g->es_off[e] + s] = lse_t(sel, cnt, T);"),
    "lse_missing_temperature_scale": ("return M + T * log(s);", "return M + log(s);"),
    "lse_missing_temperature_in_exp": ("s += exp((x[i] - M) / T);", "s += exp(x[i] - M);"),
    "or_child_missing_min_term": (
        "a1 = total + (mx < 0 ? mx : 0.0);", "a1 = total;"),
    "or_parent_missing_min_term": (
        "double alt = dc + loo + (mo < 0 ? mo : 0.0);", "double alt = dc + loo;"),
    "or_parent_missing_lem": (
        "a0 = sp_t(dc + lem_t(loo, T), T);", "a0 = sp_t(dc + loo, T);"),
    "lem_is_softplus": (
        "return a + T * log(-expm1(-a / T));", "return T * log1p(exp(a / T));"),
    "or_relu_dropped": (
        "term[j] = (T == 0.0) ? (delta[j] > 0 ? delta[j] : 0.0) : sp_t(delta[j], T);",
        "term[j] = (T == 0.0) ? delta[j] : sp_t(delta[j], T);"),
    "and_without_input_negation": (
        "double sgn = flip ? -1.0 : 1.0;", "double sgn = 1.0;"),
    "and_without_output_swap": (
        "        u[o + 0] = flip ? a1 : a0;\n        u[o + 1] = flip ? a0 : a1;\n    }\n    /* parents",
        "        u[o + 0] = a0;\n        u[o + 1] = a1;\n    }\n    /* parents"),
    "leave_one_out_off_by_one": (
        "double loo = pre[i] + suf[i + 1];", "double loo = pre[i] + suf[i];"),
    "map_argmin": ("if (b[s] > b[best]) best = s;", "if (b[s] < b[best]) best = s;"),
    "q_not_normalised": ("q[g->vs_off[v] + s] = b[s] - z;", "q[g->vs_off[v] + s] = b[s];"),
    "adjoint_missing_direct_term": ("gn[o + s] -= gu;", ""),
    "adjoint_softmax_without_T": (
        "gscore[c] += gu * exp((score[c] - z) / T);", "gscore[c] += gu * exp(score[c] - z);"),
    "adjoint_readout_without_softmax": (
        "gB[g->vs_off[v] + s] = gq[g->vs_off[v] + s] - exp((b[s] - z) / T) * tot;",
        "gB[g->vs_off[v] + s] = gq[g->vs_off[v] + s];"),
    "adjoint_damping_swapped": ("gm[i] = d * gmp[i];", "gm[i] = (1.0 - d) * gmp[i];"),
    "adjoint_vtof_sign": (
        "gm[g->es_off[e] + s] -= gn[g->es_off[e] + s];",
        "gm[g->es_off[e] + s] += gn[g->es_off[e] + s];"),
    "residual_always_zero": ("double a = fabs(mn[i] - m[i]);", "double a = 0.0;"),
    "residual_of_state_not_change": ("double a = fabs(mn[i] - m[i]);", "double a = fabs(mn[i]);"),
}


def _checks(P):
    """(name, callable) pins run against every build."""
    return [
        ("tree0", lambda: P.test_tree_exact_marginals(0, 0.0)),
        ("tree1", lambda: P.test_tree_exact_marginals(1, 0.7)),
        ("tree3", lambda: P.test_tree_exact_marginals(3, 1.0)),
        ("tree4", lambda: P.test_tree_exact_marginals(4, 0.05)),
        ("chain", lambda: P.test_chain_exact(1.0)),
        ("or0", lambda: P.test_logical_closed_form_vs_enumeration(P.W.OR, 3, 0.0)),
        ("or03", lambda: P.test_logical_closed_form_vs_enumeration(P.W.OR, 3, 0.3)),
        ("and0", lambda: P.test_logical_closed_form_vs_enumeration(P.W.AND, 3, 0.0)),
        ("off0", lambda: P.test_logical_all_parents_off(0.0)),
        ("off1", lambda: P.test_logical_all_parents_off(1.0)),
        ("and1", lambda: P.test_logical_closed_form_vs_enumeration(P.W.AND, 3, 1.0)),
        ("damped", lambda: P.test_damped_step_vs_enumeration(0.5, 0.3)),
        ("enum_dense", lambda: P.test_enum_factor_vs_enumeration((3, 3, 2), False)),
        ("enum_expl", lambda: P.test_enum_factor_vs_enumeration((3, 3, 2), True)),
        ("gauge", lambda: P.test_gauge_invariance(1.0)),
        ("evidence", P.test_zero_iterations_gives_normalised_evidence),
        ("adjoint_fd", lambda: P.test_adjoint_vs_finite_differences(True, 1.0)),
        ("adjoint_fd_T", lambda: P.test_adjoint_vs_finite_differences(False, 0.5)),
        ("adjoint_fd_d", lambda: P.test_adjoint_fd_damping(0.3)),
        ("adjoint_tree", P.test_adjoint_tree_closed_form),
        ("resid0", lambda: P.test_residual_history_matches_separate_runs(0.0)),
    ]


def _build(tmp_path, name, src_text):
    c = tmp_path / (name + ".c")
    so = tmp_path / ("lib" + name + ".so")
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", str(c),
                           "-o", str(so), "-lm"])
    return str(so)


def _failing_checks(lib):
    """Runs the checks in a child process (a planted mistake may crash the
    oracle); a crash counts as caught."""
    r = subprocess.run([sys.executable, os.path.abspath(__file__), lib], capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return ["crash(%d)" % r.returncode]
    return [x for x in r.stdout.split() if x]


def test_unmutated_source_passes(tmp_path):
    src = open(SRC).read()
    assert _failing_checks(_build(tmp_path, "orig", src)) == []


@pytest.mark.parametrize("mutation", sorted(MUTATIONS))
def test_mutation_is_caught(mutation, tmp_path):
    old, new = MUTATIONS[mutation]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found once: %s" % mutation
    lib = _build(tmp_path, mutation, src.replace(old, new))
    failed = _failing_checks(lib)
    assert failed, "no pin caught the planted mistake %s" % mutation


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path[:0] = [here, os.path.dirname(here)]
    import test_oracle_pins as P
    from oracle import OracleGraph

    P.OracleGraph = lambda g: OracleGraph(g, lib_path=sys.argv[1])
    for name, fn in _checks(P):
        try:
            fn()
        except (AssertionError, RuntimeError, FloatingPointError):
            print(name)
