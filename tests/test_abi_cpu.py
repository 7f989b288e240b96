"""Host-only checks of the C-ABI: the library loads, exports every symbol the
header declares, and validation returns the documented error codes (no GPU
call is made)."""
import os
import re

import numpy as np
import pytest

from paper_2202_04110_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbp():
    from paper_2202_04110_amd import lbp as mod
    return mod


def test_exports_every_declared_symbol(lbp):
    hdr = open(os.path.join(ROOT, "include", "lbp.h")).read()
    declared = set(re.findall(r"\b(lbp_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    missing = [s for s in sorted(declared) if not hasattr(lbp._lib, s)]
    assert not missing, missing


def test_validate_sizes(lbp):
    for g in (W.ising_grid(8, 1), W.potts_grid(5, 3, 2), W.rbm(7, 5, 3),
              W.random_factor_graph(3, 9, tree=False, extra_factors=4, logical_frac=0.3),
              W.deconv(seed=4, K=2, tw=3, sd=5, img=6)):
        s = lbp.validate(g)
        assert s == {"V": g.num_vars, "VS": g.num_var_states, "F": g.num_factors, "E": g.num_edges,
                     "ES": g.num_edge_states, "Tn": g.num_logpots}


def _expect(lbp, g, code, match=None):
    with pytest.raises(lbp.LBPError) as ei:
        lbp.validate(g)
    assert ei.value.code == code, str(ei.value)
    if match:
        assert re.search(match, str(ei.value)), str(ei.value)


def test_validation_errors(lbp):
    base = W.random_factor_graph(8, 8, tree=False, extra_factors=3, logical_frac=0.3, explicit_frac=0.5)
    E = lbp.LBP_E_INVALID

    g = base.copy(); g.edge_var[0] = g.num_vars
    _expect(lbp, g, E, "edge_var")
    g = base.copy(); g.edge_var[0] = -1
    _expect(lbp, g, E, "edge_var")
    g = base.copy(); g.factor_edge_off[1], g.factor_edge_off[2] = g.factor_edge_off[2], g.factor_edge_off[1]
    _expect(lbp, g, E)
    g = base.copy(); g.factor_edge_off[0] = 1
    _expect(lbp, g, E, "factor_edge_off")
    g = base.copy(); g.var_num_states[0] = 1
    _expect(lbp, g, E, "var_num_states")
    g = base.copy(); g.var_num_states[0] = 65
    _expect(lbp, g, E, "var_num_states")
    g = base.copy(); g.evidence[3] = np.nan
    _expect(lbp, g, E, "evidence")
    g = base.copy()
    if g.num_logpots:
        g.log_potentials[0] = np.inf
        _expect(lbp, g, E, "log_potentials")
    g = base.copy(); g.factor_kind[0] = 7
    _expect(lbp, g, E, "factor_kind")


def test_logical_needs_binary_and_parent(lbp):
    g = W.single_logical(1, W.OR, 3)
    g.var_num_states[0] = 3
    g.evidence = np.zeros(g.num_var_states, np.float32)
    _expect(lbp, g, lbp.LBP_E_INVALID, "non-binary")
    g = W.single_logical(1, W.AND, 1)
    g.factor_edge_off[1] = 1
    g.edge_var = g.edge_var[:1]
    _expect(lbp, g, lbp.LBP_E_INVALID, "parent")


def test_table_checks(lbp):
    g = W.single_enum(3, (2, 3), explicit=True)
    # a configuration state out of range for its variable
    bad = g.copy(); bad.cfg_table_states[1] = 5
    _expect(lbp, bad, lbp.LBP_E_INVALID, "out of range")
    # drop every configuration that has slot 1 in state 2 -> uncovered state
    cfg = g.cfg_table_states.reshape(-1, 2)
    keep = cfg[:, 1] != 2
    bad = g.copy()
    bad.cfg_table_states = cfg[keep].reshape(-1)
    bad.cfg_table_num_cfgs[0] = int(keep.sum())
    bad.cfg_table_off[1] = bad.cfg_table_states.shape[0]
    bad.log_potentials = bad.log_potentials[: int(keep.sum())]
    bad.logpot_off[1] = int(keep.sum())
    _expect(lbp, bad, lbp.LBP_E_INVALID, "no configuration")
    # wrong log-potential count
    bad = g.copy(); bad.logpot_off[1] -= 1; bad.log_potentials = bad.log_potentials[:-1]
    _expect(lbp, bad, lbp.LBP_E_INVALID, "log-potentials")
    # table arity differs from the factor's
    bad = g.copy(); bad.cfg_table_arity[0] = 3
    _expect(lbp, bad, lbp.LBP_E_INVALID)


def test_unsupported_limits(lbp):
    # a logical factor beyond 1024 edges
    g = W.single_logical(1, W.OR, 1100)
    _expect(lbp, g, lbp.LBP_E_UNSUPPORTED)
    # a dense 3-ary factor of 20-state variables: 8000 configurations
    g = W.single_enum(1, (20, 20, 20))
    _expect(lbp, g, lbp.LBP_E_UNSUPPORTED)


def test_empty_graph_validates(lbp):
    g = W.disjoint_union([])
    assert lbp.validate(g) == {"V": 0, "VS": 0, "F": 0, "E": 0, "ES": 0, "Tn": 0}


def test_context_without_gpu_reports_error(lbp):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import ctypes as C
    h = C.c_void_p(12345)
    rc = lbp._lib.lbp_ctx_create(0, None, C.byref(h))
    assert rc in (lbp.LBP_E_HIP, lbp.LBP_E_INVALID)
    assert h.value == 12345  # out-parameter untouched
    assert lbp.last_error()


def test_null_handles_are_rejected(lbp):
    """Every entry point taking a handle rejects NULL with LBP_E_INVALID
    (no GPU needed) and leaves out-parameters untouched."""
    import ctypes as C
    L = lbp._lib
    out = C.c_void_p(777)
    n = C.c_int32(5)
    f = C.c_float(2.5)
    for rc in (L.lbp_run_bp(None, 1, 0.5, 1.0),
               L.lbp_run_bp_until(None, 10, 0.5, 1.0, 1e-3, 1, C.byref(n), C.byref(f)),
               L.lbp_sampler_create(None, 4, C.byref(out)),
               L.lbp_sampler_run(None, 1, 0.5, 0.0, None, None, None),
               L.lbp_batch_run(None, 1, 0.5, 1.0),
               L.lbp_batch_use_fused(None, 1),
               L.lbp_batch_autotune(None, 0.5, 1.0, 3, C.byref(n)),
               L.lbp_graph_num_launches(None, C.byref(n)),
               L.lbp_graph_use_fused(None, 1),
               L.lbp_graph_use_resident(None, 1),
               L.lbp_graph_resident_state(None, None),
               L.lbp_reset_messages(None),
               L.lbp_run_bp_record(None, 5, 0.5, 1.0, 2),
               L.lbp_graph_set_fused_launch(None, 0, 4, 2),
               L.lbp_server_submit_until(None, None, 10, 0.5, 1.0, 1e-3, 5, -1.0, 1)):
        assert rc == lbp.LBP_E_INVALID
    assert out.value == 777 and n.value == 5 and f.value == 2.5
    L.lbp_sampler_free(None)
    L.lbp_batch_free(None)


def _layout_cases():
    import test_gpu_parity as T
    cases = [(n, mk) for n, mk, _ in T.STEP_CASES]
    cases += [("potts512", lambda: W.potts_grid(512, 5, 2)), ("rbm", lambda: W.rbm(784, 500, 3)),
              ("deconv", lambda: W.deconv(seed=4)), ("empty", lambda: W.disjoint_union([])),
              ("union", lambda: W.disjoint_union([W.potts_grid(5, 8, 1), W.ising_grid(3, 2),
                                                  W.single_logical(3, W.AND, 200)])),
              ("single_var", lambda: W._general_graph(np.array([7], np.int32),
                                                      np.zeros(7, np.float32), [], "one"))]
    return cases


@pytest.mark.parametrize("name", [c[0] for c in _layout_cases()])
def test_layout_bounds(lbp, name):
    """Every kernel address lands inside its array, for every test shape."""
    mk = dict(_layout_cases())[name]
    info = lbp.check_layout(mk())
    assert info["M"] > 0 and info["VB"] > 0


def test_compile_reports_first_nonfinite_potential(lbp):
    """Compilation checks the log-potentials while it copies them into their
    panels: the first non-finite entry is named, whatever the tile order."""
    g = W.random_factor_graph(11, num_vars=40, tree=False, extra_factors=30, max_arity=3, explicit_frac=0.4)
    n = g.num_logpots
    assert n > 20
    for idx in (n - 1, n // 2, 3):
        h = g.copy()
        h.log_potentials[idx] = np.nan
        h.log_potentials[n - 1] = -np.inf if idx != n - 1 else np.nan
        with pytest.raises(lbp.LBPError) as ei:
            lbp.check_layout(h)
        assert ei.value.code == lbp.LBP_E_INVALID
        assert "log_potentials[%d]" % idx in str(ei.value)
    lbp.check_layout(g)  # the clean graph compiles
