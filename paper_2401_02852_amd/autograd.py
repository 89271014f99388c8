"""torch.autograd.Function over the library's forward and adjoint gradient.

    p_succ, e_cost = QAOAFunction.apply(gammas, betas, cost, n, m)

gammas and betas are float64 tensors of length p (any device; they are read on
the host). The backward pass calls qnae_qaoa_grad with the incoming
gradients as the weights: for F = g_p * p_succ + g_E * E[C], dF/dtheta is
exactly the vector-Jacobian product autograd asks for.
"""
from __future__ import annotations

import torch

from ._binding import qaoa_grad, qaoa_run


class QAOAFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gammas, betas, cost, n: int, m: int, checkpoint_every: int = 4, context=None):
        g = gammas.detach().to("cpu", torch.float64).numpy()
        b = betas.detach().to("cpu", torch.float64).numpy()
        r = qaoa_run(cost, n, m, g, b, ctx=context)
        ctx.save_for_backward(gammas, betas)
        ctx.cost, ctx.n, ctx.m, ctx.every, ctx.context = cost, n, m, checkpoint_every, context
        return (torch.tensor(r.p_success, dtype=torch.float64, device=gammas.device),
                torch.tensor(r.expected_cost, dtype=torch.float64, device=gammas.device))

    @staticmethod
    def backward(ctx, grad_p, grad_e):
        gammas, betas = ctx.saved_tensors
        wp = float(grad_p) if grad_p is not None else 0.0
        we = float(grad_e) if grad_e is not None else 0.0
        dg, db, _ = qaoa_grad(ctx.cost, ctx.n, ctx.m, gammas.detach().cpu().numpy(),
                              betas.detach().cpu().numpy(), w_psucc=wp, w_energy=we,
                              checkpoint_every=ctx.every, ctx=ctx.context)
        return (torch.from_numpy(dg).to(gammas.device, gammas.dtype),
                torch.from_numpy(db).to(betas.device, betas.dtype), None, None, None, None, None)
