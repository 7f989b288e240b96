"""torch.autograd.Function over the library's record / backward calls.

Differentiates the normalised beliefs of damped sum-product LBP (T > 0) with
respect to the log-potentials and the evidence: the paper's use of LBP "as
part of a larger end-to-end differentiable system" (Sec. "Exciting new
possibilities from implementing LBP in JAX").  The forward pass runs the
solver with checkpoints every ``ckpt_every`` iterations; the backward pass is
the library's reverse sweep (HIP kernels), not torch autodiff.
"""
from __future__ import annotations

import torch


class LBPBeliefs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_potentials, evidence, graph, iters, damping, temperature, ckpt_every):
        graph.set_log_potentials(log_potentials.detach().contiguous().float())
        graph.set_evidence(evidence.detach().contiguous().float())
        graph.reset_messages()
        graph.run_bp_record(iters, damping, temperature, ckpt_every)
        q = torch.empty(graph.VS, device=evidence.device, dtype=torch.float32)
        graph.get_beliefs(out=q)
        ctx.graph = graph
        return q

    @staticmethod
    def backward(ctx, grad_q):
        g = ctx.graph
        dev = grad_q.device
        gphi = torch.empty(g.Tn, device=dev, dtype=torch.float32)
        gth = torch.empty(g.VS, device=dev, dtype=torch.float32)
        g.backward(grad_q.detach().contiguous().float(), gphi, gth)
        return gphi, gth, None, None, None, None, None


def lbp_beliefs(graph, log_potentials, evidence, iters: int, damping: float = 0.5,
                temperature: float = 1.0, ckpt_every: int = 10):
    """Normalised beliefs q (flat, variable-major) as a differentiable function
    of ``log_potentials`` (Tn) and ``evidence`` (VS), both device tensors."""
    return LBPBeliefs.apply(log_potentials, evidence, graph, int(iters), float(damping),
                            float(temperature), int(ckpt_every))
