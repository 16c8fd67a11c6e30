"""``torch.autograd.Function`` over the HIP forward and adjoint.

``EdgeMetrics.apply(coords, topo, elems, reduce)`` returns ``(n, b, V)`` (the
lumped directed-area vectors, boundary dual-face normals and element-based
dual volumes) and back-propagates through ``eb_directed_areas_backward``:
dL/dx from dL/dn, dL/db and dL/dV, with each element's orientation held
fixed (the metrics are polynomials in x away from degenerate elements).
"""
from __future__ import annotations

import torch

from . import api

__all__ = ["EdgeMetrics", "edge_metrics"]


class EdgeMetrics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, topo, elems, reduce="gather"):
        n, b, V = api.directed_areas(coords.detach(), topo, elems, reduce=reduce)
        ctx.save_for_backward(coords)
        ctx.topo, ctx.elems, ctx.reduce = topo, elems, reduce
        return n, b, V

    @staticmethod
    def backward(ctx, gn, gb, gV):
        (coords,) = ctx.saved_tensors
        def c(t):
            return None if t is None else t.contiguous()
        g = api.directed_areas_backward(coords.detach(), ctx.topo, ctx.elems, c(gn), c(gb),
                                        c(gV), reduce=ctx.reduce)
        return g, None, None, None


def edge_metrics(coords, topo, elems, reduce="gather"):
    return EdgeMetrics.apply(coords, topo, elems, reduce)
