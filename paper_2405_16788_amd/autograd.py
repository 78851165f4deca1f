"""Differentiation pattern: the dipole-sum query as a torch.autograd.Function.

Forward evaluates the Barnes-Hut sums (values and spatial gradients) with
``dps_query``; backward runs the two-stage adjoint of Sec. 6.2 / App. C
(``dps_adjoint``: node accumulation with a recomputed traversal, then the
push-down to the points).  Nothing about the traversal is stored between the
two passes: the adjoint walks the tree again for each query.

The value D(x) is linear in the attributes, and the traversal depends only on
x and the fixed geometry, so dL/dattrs is the exact transpose of the forward
map; dL/dx is sum_c dL/dD_c * grad_x D_c with the same accepted sources.
"""
from __future__ import annotations

import torch

from . import binding as B


def _refit_if_changed(tree: B.Tree, attrs: torch.Tensor):
    key = (attrs.data_ptr(), attrs._version)
    if getattr(tree, "_attr_key", None) != key:
        B.dps_set_attributes(tree, attrs)
        tree._attr_key = key


class DipoleSum(torch.autograd.Function):
    """f, grad = DipoleSum.apply(attrs[M,C], x[Q,3], tree, beta, eps).

    ``f`` [Q,C] is differentiable w.r.t. attrs and x; ``grad`` [Q,C,3] is
    returned as a non-differentiable output."""

    @staticmethod
    def forward(ctx, attrs, x, tree, beta, eps):
        attrs_c = attrs.detach().contiguous()
        x_c = x.detach().contiguous()
        _refit_if_changed(tree, attrs_c)
        f, g = B.dps_query(tree, x_c, beta, eps, grad=True)
        ctx.save_for_backward(x_c, attrs_c)
        ctx.tree, ctx.beta, ctx.eps = tree, float(beta), float(eps)
        ctx.mark_non_differentiable(g)
        return f, g

    @staticmethod
    def backward(ctx, df, dg):
        if dg is not None and bool(torch.any(dg != 0)):
            raise NotImplementedError("cotangents of the spatial gradient output are not supported")
        x, attrs = ctx.saved_tensors
        tree = ctx.tree
        _refit_if_changed(tree, attrs)
        need_attr, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if df is None or not (need_attr or need_x):
            return None, None, None, None, None
        dattrs, dx = B.dps_adjoint(tree, x, ctx.beta, ctx.eps, df.contiguous().to(torch.float32),
                                   want_dx=need_x)
        dattrs = dattrs.reshape(attrs.shape) if need_attr else None
        return dattrs, (dx if need_x else None), None, None, None


def dipole_sum(attrs, x, tree, beta: float, eps: float):
    """Functional form of ``DipoleSum``: returns (f, grad)."""
    return DipoleSum.apply(attrs, x, tree, beta, eps)
