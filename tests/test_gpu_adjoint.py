"""Reverse sweep (HIP, through the C-ABI) against the FP64 oracle's reverse
mode, on the same seeded graphs.

Tolerance: |g_gpu - g_oracle| <= 2e-4 * max(1, max|g_oracle|) on every entry
of dL/dphi and dL/dtheta (FP32 reverse sweep over tens of iterations; the
oracle's gradient is itself pinned to finite differences and to the tree
closed form in test_oracle_pins.py).
"""
import os

import numpy as np
import pytest

from oracle import OracleGraph
from paper_2202_04110_amd import workloads as W

pytestmark = pytest.mark.gpu
NT = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def lbp(gpu_lib):
    return gpu_lib


@pytest.fixture(scope="module")
def ctx(lbp):
    return lbp.Context(0)


def gpu_grad(lbp, ctx, spec, iters, d, T, gq, k):
    import torch
    g = lbp.Graph(ctx, spec)
    g.run_bp_record(iters, d, T, k)
    gphi = torch.empty(g.Tn, device="cuda", dtype=torch.float32)
    gth = torch.empty(g.VS, device="cuda", dtype=torch.float32)
    g.backward(torch.from_numpy(gq.astype(np.float32)).cuda(), gphi, gth)
    torch.cuda.synchronize()
    return g, gphi.cpu().numpy(), gth.cpu().numpy()


def check(spec, ga, gb, label):
    oa, ob = ga
    pa, pb = gb
    scale = max(1.0, float(np.abs(oa).max()) if oa.size else 1.0, float(np.abs(ob).max()))
    ea = float(np.abs(pa - oa).max()) if oa.size else 0.0
    eb = float(np.abs(pb - ob).max())
    print("%s: max|dphi err| %.2e, max|dtheta err| %.2e, scale %.2f" % (label, ea, eb, scale))
    assert ea <= 2e-4 * scale and eb <= 2e-4 * scale


def small_graphs():
    return [
        ("tree", W.random_factor_graph(31, num_vars=9, tree=True, max_arity=3, explicit_frac=0.4, lp_sd=0.7)),
        ("loopy", W.random_factor_graph(32, num_vars=12, tree=False, extra_factors=8, max_arity=3,
                                        explicit_frac=0.4, lp_sd=0.7)),
        ("potts10x4", W.potts_grid(10, 4, seed=5)),
        ("potts9x3", W.potts_grid(9, 3, seed=6)),
        ("rect", W.disjoint_union([W.potts_grid(6, 2, 1), W.potts_grid(5, 7, 2)])),
        ("triplet7x3", W.triplet_grid(7, 3, 9)),
        ("layer70x80", layer(10, 70, 80)),
    ]


def layer(seed, nv, nh, drop=0.03):
    """A bipartite layer of binary units with about 3% of its factors missing:
    every unit has more than 64 edges, so the hidden units sum their messages
    in column groups in the recorded forward sweep."""
    rng = np.random.default_rng(seed)
    i, j = np.nonzero(rng.random((nv, nh)) >= drop)
    pairs = np.stack([i, nv + j], 1).astype(np.int64)
    ev = rng.normal(0, 0.5, (nv + nh) * 2).astype(np.float32)
    tab = rng.normal(0, 0.3, (pairs.shape[0], 4)).astype(np.float32)
    return W._pairwise_graph(np.full(nv + nh, 2, np.int32), ev, pairs, tab, "layer%dx%d" % (nv, nh))


@pytest.mark.parametrize("idx", range(7))
@pytest.mark.parametrize("T,d", [(1.0, 0.5), (0.5, 0.3)])
def test_adjoint_matches_oracle(lbp, ctx, idx, T, d):
    name, spec = small_graphs()[idx]
    og = OracleGraph(spec)
    gq = np.random.default_rng(idx).normal(0, 1, og.VS)
    iters = 15
    gphi_o, gth_o, _ = og.backward(iters, d, T, gq)
    _, gphi, gth = gpu_grad(lbp, ctx, spec, iters, d, T, gq, 4)
    check(spec, (gphi_o, gth_o), (gphi, gth), "%s T=%g d=%g" % (name, T, d))


def test_checkpoint_interval_does_not_change_bits(lbp, ctx):
    spec = W.potts_grid(12, 5, seed=7)
    gq = np.random.default_rng(1).normal(0, 1, spec.num_var_states)
    res = [gpu_grad(lbp, ctx, spec, 23, 0.5, 1.0, gq, k)[1:] for k in (1, 4, 10, 23, 100)]
    for gphi, gth in res[1:]:
        np.testing.assert_array_equal(gphi, res[0][0])
        np.testing.assert_array_equal(gth, res[0][1])


def test_served_shape_gradient(lbp, ctx):
    """A served-stream request shape: Potts 64x64, 6 states, 50 iterations,
    checkpoint every 10, loss sum(c * q) with c ~ N(0,1)."""
    req = {"L": 64, "n": 6, "seed": 77}
    spec = W.request_graph(req)
    gq = W.request_loss_coeffs(req).astype(np.float64)
    og = OracleGraph(spec)
    gphi_o, gth_o, _ = og.backward(50, 0.5, 1.0, gq)
    _, gphi, gth = gpu_grad(lbp, ctx, spec, 50, 0.5, 1.0, gq, 10)
    check(spec, (gphi_o, gth_o), (gphi, gth), "potts64x6 50 iters")


def test_autograd_function(lbp, ctx):
    import torch
    from paper_2202_04110_amd.autograd import lbp_beliefs
    spec = W.potts_grid(11, 3, seed=9)
    g = lbp.Graph(ctx, spec)
    phi = torch.from_numpy(spec.log_potentials.copy()).cuda().requires_grad_(True)
    th = torch.from_numpy(spec.evidence.copy()).cuda().requires_grad_(True)
    c = torch.from_numpy(np.random.default_rng(3).normal(0, 1, spec.num_var_states).astype(np.float32)).cuda()
    q = lbp_beliefs(g, phi, th, 20, 0.5, 1.0, 5)
    loss = (c * q).sum()
    loss.backward()
    og = OracleGraph(spec)
    gphi_o, gth_o, _ = og.backward(20, 0.5, 1.0, c.cpu().numpy().astype(np.float64))
    check(spec, (gphi_o, gth_o), (phi.grad.cpu().numpy(), th.grad.cpu().numpy()), "autograd")
    # forward value equals the oracle's beliefs
    _, qo, _ = og.beliefs(og.run(20, 0.5, 1.0), 1.0)
    assert np.abs(q.detach().cpu().numpy() - qo).max() < 1e-4


def test_backward_state_and_argument_errors(lbp, ctx):
    import torch
    spec = W.potts_grid(6, 3, seed=2)
    g = lbp.Graph(ctx, spec)
    gq = torch.zeros(g.VS, device="cuda")
    gp = torch.empty(g.Tn, device="cuda")
    with pytest.raises(lbp.LBPError) as ei:
        g.backward(gq, gp)
    assert ei.value.code == lbp.LBP_E_STATE
    with pytest.raises(lbp.LBPError) as ei:
        g.run_bp_record(10, 0.5, 0.0, 5)
    assert ei.value.code == lbp.LBP_E_INVALID
    g.run_bp_record(10, 0.5, 1.0, 5)
    g.backward(gq, gp)
    g.backward(gq, gp)  # the record stays valid
    g.run_bp(1, 0.5, 1.0)
    with pytest.raises(lbp.LBPError) as ei:
        g.backward(gq, gp)
    assert ei.value.code == lbp.LBP_E_STATE
    lg = lbp.Graph(ctx, W.single_logical(1, W.OR, 4))
    with pytest.raises(lbp.LBPError) as ei:
        lg.run_bp_record(5, 0.5, 1.0, 2)
    assert ei.value.code == lbp.LBP_E_UNSUPPORTED


def test_gradient_matches_finite_differences(lbp, ctx):
    """GPU dL/dphi and dL/dtheta against central differences of the FP64
    oracle's loss L = sum(gq * q(N iterations)), perturbing single float32
    inputs by +-2^-7 (exact in float32 at these magnitudes)."""
    import copy
    spec = W.random_factor_graph(33, num_vars=10, tree=False, extra_factors=6, max_arity=3,
                                 explicit_frac=0.4, lp_sd=0.7)
    iters, d, T = 12, 0.5, 1.0
    og = OracleGraph(spec)
    gq = np.random.default_rng(7).normal(0, 1, og.VS)
    _, gphi, gth = gpu_grad(lbp, ctx, spec, iters, d, T, gq, 5)

    def loss(s):
        o = OracleGraph(s)
        _, q, _ = o.beliefs(o.run(iters, d, T), T)
        return float(np.dot(gq, q))

    h = 2.0 ** -7
    rng = np.random.default_rng(8)
    scale = max(1.0, float(np.abs(gphi).max()), float(np.abs(gth).max()))
    for field, grad, picks in (("log_potentials", gphi, rng.choice(len(spec.log_potentials), 6, replace=False)),
                               ("evidence", gth, rng.choice(len(spec.evidence), 4, replace=False))):
        for i in picks:
            vals = []
            for sgn in (1.0, -1.0):
                s = copy.deepcopy(spec)
                arr = getattr(s, field).astype(np.float32).copy()
                arr[i] = np.float32(arr[i] + sgn * h)
                setattr(s, field, arr)
                vals.append(loss(s))
            fd = (vals[0] - vals[1]) / (2 * h)
            print("%s[%d]: gpu %.6f fd %.6f" % (field, i, grad[i], fd))
            assert abs(grad[i] - fd) <= 1e-3 * scale


def test_learning_loop_matches_oracle_gradient_descent(lbp, ctx):
    """Gradient descent on a marginal-matching cross-entropy through the
    reverse sweep (learn.fit) follows the trajectory of the same descent
    driven by the FP64 oracle's gradients, and lowers the loss."""
    import copy
    import torch
    from paper_2202_04110_amd.learn import fit
    spec = W.potts_grid(8, 3, seed=21)
    teacher = copy.deepcopy(spec)
    teacher.log_potentials = np.random.default_rng(22).normal(0, 1.0, len(spec.log_potentials)).astype(np.float32)
    iters, d, lr, steps = 30, 0.5, 0.5, 6
    ot = OracleGraph(teacher)
    _, qt, _ = ot.beliefs(ot.run(iters, d, 1.0), 1.0)
    target = np.exp(qt)
    g = lbp.Graph(ctx, spec)
    phi_g, _, losses = fit(g, torch.from_numpy(target.astype(np.float32)).cuda(),
                           torch.from_numpy(spec.log_potentials.copy()).cuda(),
                           torch.from_numpy(spec.evidence.copy()).cuda(), steps=steps, lr=lr, iters=iters, damping=d,
                           ckpt_every=10)
    phi_g = phi_g.cpu().numpy()
    # the same descent on the oracle's gradients (FP32 tables, as the library holds them)
    phi = spec.log_potentials.astype(np.float32).copy()
    s = copy.deepcopy(spec)
    for _ in range(steps):
        s.log_potentials = phi
        og = OracleGraph(s)
        gphi, _, _ = og.backward(iters, d, 1.0, -target / spec.num_vars)
        phi = (phi - np.float32(lr) * gphi.astype(np.float32)).astype(np.float32)
    err = float(np.abs(phi_g - phi).max())
    print("losses %s; max |phi_gpu - phi_oracle| after %d steps = %.2e" % (np.round(losses, 5), steps, err))
    assert err <= 2e-4 * max(1.0, float(np.abs(phi).max()))
    assert losses[-1] < losses[0]
