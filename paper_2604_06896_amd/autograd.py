"""Differentiable equilibrium: X* = argmin_X E(X, theta) as a torch op.

Forward relaxes the tissue with libvtx (gradient descent with T1 exchanges;
Methods, "Simulation engine").  Backward receives dL/dX* from any outer cost
and returns dL/dtheta through the library's hypergradient (Methods,
"Gradient computation methods"):
  * "adjoint": implicit differentiation, H mu = P dL/dX* by CG on the
    Hessian-vector-product kernels, then -(d2E/dX dtheta)^T mu;
  * "ep": centred equilibrium propagation with the linear nudge
    (dL/dX*) . X, i.e. two nudged relaxations at +-beta/2 from X*.
theta is either the per-edge line tensions (theta="lambda") or the per-cell
preferred perimeters (theta="P0"); the other parameters are held fixed.
"""
from __future__ import annotations

import dataclasses

import torch

from . import vtx as V


class VertexEquilibrium(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, X0, tissue, params, which, mode, relax_kw, grad_kw):
        X = X0.detach().clone().contiguous()
        prm = dataclasses.replace(params, **{("lam" if which == "lambda" else "P0"):
                                             theta.detach().to(X.dtype)})
        info = tissue.relax(X, prm, mode=mode, **relax_kw)
        ctx.tissue, ctx.prm, ctx.which, ctx.mode, ctx.grad_kw = tissue, prm, which, mode, grad_kw
        ctx.relax_info = info
        ctx.save_for_backward(X, theta)
        return X

    @staticmethod
    def backward(ctx, gX):
        X, theta = ctx.saved_tensors
        kw = dict(ctx.grad_kw)
        method = kw.pop("method", "adjoint")
        g, info = ctx.tissue.param_grad(X, ctx.prm, dC_dX=gX.to(torch.float64).contiguous(),
                                        method=method, theta=ctx.which, mode=ctx.mode, **kw)
        ctx.grad_info = info
        return g.to(theta.dtype), None, None, None, None, None, None, None


def equilibrium(theta, X0, tissue, params, which="lambda", mode="f64", relax=None, grad=None):
    """X*(theta) with a hypergradient backward.  `relax` and `grad` are
    keyword dicts for Tissue.relax and Tissue.param_grad (grad may set
    method="adjoint" or "ep")."""
    return VertexEquilibrium.apply(theta, X0, tissue, params, which, mode, relax or {},
                                   grad or {})
