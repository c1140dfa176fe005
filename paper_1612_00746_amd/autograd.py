"""torch.autograd face of the adjoint in libctqw.

``EnsembleLoss.apply(Jbar, epsbar, model)`` returns the ensemble-averaged
diagonal observable L = (1/R) sum_r <psi_r(T)|W|psi_r(T)> of a noisy walk
whose realisation r has hoppings Jbar + dJ_r and on-site energies
epsbar + deps_r (fixed noise draws held by ``model``).  The forward pass
propagates with checkpoints (``ctqw_forward_ckpt``) and evaluates the loss
(``ctqw_loss``); the backward pass recomputes each checkpoint segment and
runs the hand-written adjoint kernels (``ctqw_backward``), returning
dL/dJbar and dL/depsbar scaled by the incoming gradient.  Only argument
marshalling happens here.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import Plan


@dataclasses.dataclass
class NoisyWalk:
    """A bound plan plus the fixed noise draws and the loss definition."""
    plan: Plan
    dJ: np.ndarray          # [R, n_bonds]
    deps: np.ndarray        # [R, N]
    U: np.ndarray           # [R]
    sites: list             # start sites
    n_steps: int
    ckpt_every: int
    site_weights: np.ndarray
    kind: str = "product"   # "product" or "one_body"


class EnsembleLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Jbar: torch.Tensor, epsbar: torch.Tensor, model: NoisyWalk):
        Jb = Jbar.detach().cpu().double().numpy()
        eb = epsbar.detach().cpu().double().numpy()
        J = (Jb[None, :] + model.dJ).reshape(-1)
        eps = (eb[None, :] + model.deps).reshape(-1)
        model.plan.set_params(J, eps, model.U)
        model.plan.init_product_state(model.sites)
        model.plan.forward_ckpt(model.n_steps, model.ckpt_every)
        loss = model.plan.loss(model.site_weights, model.kind)
        ctx.model = model
        ctx.dev, ctx.dtype = Jbar.device, Jbar.dtype
        return torch.tensor(loss, dtype=torch.float64, device=Jbar.device)

    @staticmethod
    def backward(ctx, g):
        model = ctx.model
        _, gJ, gE = model.plan.backward(model.site_weights, model.kind)
        s = g.detach().double().cpu().item()
        return (torch.as_tensor(s * gJ, dtype=ctx.dtype, device=ctx.dev),
                torch.as_tensor(s * gE, dtype=ctx.dtype, device=ctx.dev), None)
