"""Differentiable SDP layer: X*(b, C) = argmin <C, X> s.t. A(X) = b, X PSD.

The forward pass is sdp_solve on the GPU; the backward pass is sdp_adjoint,
which returns the derivative of the central-path point at the final mu (the
self-adjoint Newton KKT system of eq. Newt-eps solved with C~ = dL/dX and
b~ = 0 after re-centring).  The constraint operator A is fixed data of the
layer; b and C are the differentiable inputs (CUDA, float64, C symmetric).
"""
from __future__ import annotations

import torch

from .api import Context


class SDPLayer(torch.autograd.Function):
    """Usage: X = SDPLayer.apply(b, C, problem, options) with options a dict of sdp_options fields.

    ``problem`` holds the fixed constraint data: {"kind": "dense", "n", "m", "A"}
    or {"kind": "entry", "n", "m", "jk"} (numpy arrays or CUDA tensors).  The
    backward pass may use a different inner precision: options["adjoint_inner_prec"].
    """

    @staticmethod
    def forward(ctx, b: torch.Tensor, C: torch.Tensor, problem: dict, options: dict | None = None):
        opts = dict(options or {})
        adj_prec = opts.pop("adjoint_inner_prec", None)
        p = dict(problem)
        p["b"] = b.detach().to(dtype=torch.float64).contiguous()
        p["C"] = C.detach().to(dtype=torch.float64).contiguous()
        if not isinstance(p.get("A", p.get("jk")), torch.Tensor):
            # host constraint data: pass b and C through the host as well
            p["b"] = p["b"].cpu().numpy()
            p["C"] = p["C"].cpu().numpy()
        sctx = Context(p, **opts)
        sctx.solve()
        X, _, _ = sctx.get_point()
        ctx.sdp = sctx
        if adj_prec is not None and adj_prec != sctx.options.inner_prec:
            # a second context for the backward pass in its own precision, at the same point
            q = dict(p)
            bopts = dict(opts)
            bopts["inner_prec"] = adj_prec
            actx = Context(q, **bopts)
            actx.set_point(*sctx.get_point())
            ctx.sdp = actx
            sctx.close()
        return X.clone()

    @staticmethod
    def backward(ctx, grad_X: torch.Tensor):
        sctx = ctx.sdp
        gb, gC, _ = sctx.adjoint(grad_X)
        sctx.close()
        ctx.sdp = None
        return gb, gC, None, None
