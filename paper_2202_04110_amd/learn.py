"""Learning factor tables with the reverse sweep: gradient descent on the
cross-entropy between target marginals and the model's sum-product beliefs.

This is LBP used inside an end-to-end differentiable objective, the use the
paper opens up (Sec. "Exciting new possibilities from implementing LBP in
JAX"): every step runs the damped sum-product solver with checkpoints
(forward), the library's reverse sweep (HIP kernels) for dL/dphi and
dL/dtheta, and a plain gradient step in torch.
"""
from __future__ import annotations

import torch

from .autograd import lbp_beliefs


def cross_entropy(q, target, num_vars: int):
    """-(1/V) sum_v sum_s p*_v(s) log b_v(s): q are the normalised log-beliefs
    at temperature 1 (log-marginals), target the marginals p*, both flat
    variable-major."""
    return -(target * q).sum() / num_vars


def fit(graph, target, log_potentials, evidence, steps: int = 20, lr: float = 0.5, iters: int = 30,
        damping: float = 0.5, ckpt_every: int = 10, fit_evidence: bool = False):
    """Runs `steps` gradient steps from (log_potentials, evidence) (device
    tensors, flat orders) towards the target marginals; returns the fitted
    tables (and evidence) and the loss before each step."""
    phi = log_potentials.detach().clone().float().requires_grad_(True)
    th = evidence.detach().clone().float().requires_grad_(fit_evidence)
    losses = []
    for _ in range(steps):
        q = lbp_beliefs(graph, phi, th, iters, damping, 1.0, ckpt_every)
        loss = cross_entropy(q, target, graph.V)
        losses.append(float(loss.detach()))
        loss.backward()
        with torch.no_grad():
            phi -= lr * phi.grad
            phi.grad = None
            if fit_evidence:
                th -= lr * th.grad
                th.grad = None
    return phi.detach(), th.detach(), losses
