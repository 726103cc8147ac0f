"""Differentiable DSC for dictionary learning over the LiFE encoding.

``y = M(D) w`` (eq. 1 with M_v = D Phi_v, eq. 3) is linear in both the
dictionary D and the weights w, so its backward pass is two products of the
library: for an upstream gradient ybar,

* dL/dw = M^T ybar                      (life_wc, the WC of the SBB step, eq. 6)
* dL/dD[:, a] = sum over nonzeros c with atom_c = a of phi_c w[f_c] ybar[:, v_c]
                                         (life_dict_grad)

The paper fits w only (SBB-NNLS); this module lets the same plan serve a loss
that also learns D, e.g. ``||y_obs - M(D) w||^2`` (``loss``).  Every product
runs in liblife.so; torch only carries the tensors.
"""
from __future__ import annotations

import torch

from . import life

__all__ = ["dsc", "loss"]


class _DSC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D, w, plan):
        ctx.plan = plan
        ctx.save_for_backward(D, w)
        return plan.dsc(D, w)

    @staticmethod
    def backward(ctx, gy):
        D, w = ctx.saved_tensors
        gy = gy.contiguous().float()
        gD = ctx.plan.dict_grad(w, gy).reshape(D.shape) if ctx.needs_input_grad[0] else None
        gw = ctx.plan.wc(D, gy) if ctx.needs_input_grad[1] else None
        return gD, gw, None


def dsc(plan: "life.Plan", D: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """y = M(D) w, differentiable in D (shape (n_atoms, n_theta) or flat) and w."""
    return _DSC.apply(D, w, plan)


def loss(plan: "life.Plan", D: torch.Tensor, w: torch.Tensor, y_obs: torch.Tensor) -> torch.Tensor:
    """L = ||y_obs - M(D) w||^2 (no 1/2)."""
    r = dsc(plan, D, w) - y_obs
    return torch.dot(r, r)
