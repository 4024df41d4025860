"""Gradients of the wetting observables of an IB-LB run for torch.autograd.

``contact_observables(params, ...)`` runs a droplet simulation through the
library and returns the height h and the signed squared contact radius r2 of
the contact-angle sphere fit as a float64 tensor; its backward pass is the
library's hand-written discrete adjoint (iblb_adjoint_record / _backward,
recomputing each checkpoint segment) and the host-side gradient of the fit.
params = (abar, k_V, eps_lo, tau) with alpha = abar * model.  Argument
marshalling only: every step and every derivative is computed by libiblb.
"""
from __future__ import annotations

import dataclasses

import torch

from . import iblb


class _ContactRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, spec):
        domain, mesh, model, steps, every, precision = spec
        abar, kv, eps, tau = (float(v) for v in params.detach().cpu())
        dom = dataclasses.replace(domain, tau=tau)
        m = dataclasses.replace(mesh, alpha=tuple(abar * k for k in model), k_v=kv, eps_wall_lo=eps)
        sim = iblb.Simulation(dom, m, precision=precision)
        sim.adjoint_record(steps, every)
        h, r2, dh, dr2 = iblb.sphere_fit_grad(sim.vertices(), 0, dom.z_lo, m.r_cut_wall)
        ctx.sim, ctx.dh, ctx.dr2, ctx.model = sim, dh, dr2, model
        return torch.tensor([h, r2], dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        dJdq = float(gout[0]) * ctx.dh + float(gout[1]) * ctx.dr2
        g, _ = ctx.sim.adjoint_backward(dJdq)  # the context lives as long as the graph (retain_graph)
        dabar = sum(mk * g[k] for k, mk in enumerate(ctx.model))
        return torch.tensor([dabar, g[3], g[4], g[5]], dtype=torch.float64), None


def contact_observables(params: torch.Tensor, domain, mesh, model, steps: int, every: int = 0,
                        precision: int = iblb.FP32_DEV) -> torch.Tensor:
    """(h, r2) after `steps` steps; differentiable with respect to params =
    (abar, k_V, eps_lo, tau).  every = 0 keeps every time level in device
    memory (no recompute); every > 0 keeps a checkpoint every `every` steps
    and recomputes each segment in the backward pass."""
    return _ContactRun.apply(params, (domain, mesh, model, steps, every, precision))
