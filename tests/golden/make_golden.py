"""Writes the stored expected values under tests/golden/ (one JSON file per
case) with the FP64 oracle and nothing else: each file holds the graph's flat
arrays, the run's parameters, the section of the paper that defines what is
computed, and the oracle's normalised log-beliefs q, MAP decode and final
residual.  Test infrastructure: run from the repository root as
``python tests/golden/make_golden.py``.  The stored values are pinned to the
mathematics in tests/test_golden.py (tree cases against brute-force
enumeration, loopy cases against the fixed-point property of a converged run)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import OracleGraph  # noqa: E402
from paper_2202_04110_amd import workloads as W  # noqa: E402

ARRAYS = ("var_num_states", "evidence", "factor_kind", "factor_edge_off", "edge_var", "factor_cfg_table",
          "cfg_table_num_cfgs", "cfg_table_arity", "cfg_table_off", "cfg_table_states", "logpot_off",
          "log_potentials")

FLAT = 'Sec. "A fully flat array-based LBP implementation"'
ENUM = 'Sec. "Specifying complex factor graphs" (enumeration factors by their valid configurations)'
LOGIC = 'Sec. "Package features" (OR/AND logical factors, damping)'

# name, graph, iterations, damping, temperature, tree?, citation
CASES = [
    ("chain5_sum", lambda: W.chain(301, 5, 3), 100, 0.5, 1.0, True, FLAT),
    ("chain6_max", lambda: W.chain(302, 6, 4), 100, 0.5, 0.0, True, FLAT),
    ("tree_explicit_t07", lambda: W.random_factor_graph(303, num_vars=7, tree=True), 100, 0.5, 0.7, True, ENUM),
    ("or4_sum", lambda: W.single_logical(304, W.OR, 4), 80, 0.5, 1.0, True, LOGIC),
    ("and5_max", lambda: W.single_logical(305, W.AND, 5), 80, 0.5, 0.0, True, LOGIC),
    ("triple_sum", lambda: W.single_enum(306, [3, 2, 4]), 80, 0.5, 1.0, True, ENUM),
    ("ising4_loopy_sum", lambda: W.ising_grid(4, 307), 300, 0.5, 1.0, False, FLAT),
    ("potts3_loopy_t05", lambda: W.potts_grid(3, 3, 308), 300, 0.5, 0.5, False, FLAT),
]


def write_case(name, make, iters, d, T, tree, cite):
    g = make()
    og = OracleGraph(g)
    m, res = og.run(iters, d, T, residuals=True)
    _, q, mp = og.beliefs(m, T)
    doc = {"name": name, "citation": cite, "tree": tree, "iters": iters, "damping": d, "temperature": T,
           "graph": {k: np.asarray(getattr(g, k)).tolist() for k in ARRAYS},
           "q": [float(x) for x in q], "map": [int(x) for x in mp], "final_residual": float(res[-1])}
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")


def main():
    for c in CASES:
        write_case(*c)
        print("wrote", c[0])


if __name__ == "__main__":
    main()
