"""Differentiation pattern: the dipole-sum query as a torch.autograd.Function.

Forward evaluates the Barnes-Hut sums (values and, optionally, spatial
gradients) with ``dps_query`` / ``dps_query_channels``; backward runs the
two-stage adjoint of Sec. 6.2 / App. C (node accumulation with a recomputed
traversal, then the push-down to the points).  Nothing about the traversal is
stored between the two passes: the adjoint walks the tree again for each query.
When the forward computed the spatial gradients, the backward forms dL/dx
from them (``dps_adjoint_accumulate_from_forward``) and its walk only
accumulates the attribute derivatives.

The value D(x) and its gradient are linear in the attributes, and the
traversal depends only on x and the fixed geometry, so dL/dattrs is the exact
transpose of the forward map; dL/dx is sum_c dL/dD_c * grad_x D_c plus, for
cotangents of the gradient output, the Hessian of D_c applied to them, with
the same accepted sources.

Both passes are free of host synchronisation, so a forward + backward built
from these calls can be captured in a graph and replayed; ``refit=True`` puts
the moment refit inside the captured work (attributes updated in place between
replays are then picked up).
"""
from __future__ import annotations

import torch

from . import binding as B


def _refit_if_changed(tree: B.Tree, attrs: torch.Tensor):
    key = (attrs.data_ptr(), attrs._version)
    if getattr(tree, "_attr_key", None) != key:
        B.dps_set_attributes(tree, attrs)
        tree._attr_key = key


def _refit(tree: B.Tree, attrs: torch.Tensor, mode):
    if mode is True:
        B.dps_set_attributes(tree, attrs)
        tree._attr_key = (attrs.data_ptr(), attrs._version)
    elif mode == "auto":
        _refit_if_changed(tree, attrs)


class DipoleSum(torch.autograd.Function):
    """f, grad = DipoleSum.apply(attrs[M,C], x[Q,3], normals, eps, tree, beta, opts).

    For a monopole-kernel tree (appearance channels) f is differentiable and
    grad is returned but carries no derivatives (no cotangents of it), and
    neither normals nor eps may be differentiated.

    ``opts`` = (c_begin, n_channels, q_count, want_grad, refit) with
    n_channels None meaning all channels.  ``f`` [Q,n] and ``grad`` [Q,n,3]
    (or None) are both differentiable w.r.t. attrs and x: cotangents of grad
    go through the Hessian adjoint (``dps_adjoint_accumulate_grad``).
    ``normals`` is None (the tree's normals) or an [M,3] tensor that replaces
    them (the moments are refitted) and is differentiable; ``eps`` is a float
    or a tensor, differentiable when it requires grad (its value is read on the
    host).  With a device row count ``q_count`` (int64 CUDA tensor [1]) only
    the first min(Q, q_count) rows are evaluated; the other rows of f / grad
    and of the position gradient are zero."""

    @staticmethod
    def forward(ctx, attrs, x, normals, eps, tree, beta, opts):
        c_begin, n_ch, q_count, want_grad, refit = opts
        ctx.set_materialize_grads(False)
        if getattr(tree, "kernel", "dipole") == "monopole" and (
                normals is not None or (isinstance(eps, torch.Tensor) and eps.requires_grad)):
            raise ValueError("normal and eps derivatives are defined for dipole-kernel trees only")
        eps_v = float(eps.detach()) if isinstance(eps, torch.Tensor) else float(eps)
        attrs_c = attrs.detach().contiguous()
        x_c = x.detach().contiguous()
        if normals is not None:
            B.dps_set_normals(tree, normals.detach().contiguous())
            refit = True  # the moments hold A n mu
        _refit(tree, attrs_c, refit)
        full = n_ch is None and q_count is None
        if full:
            f, g = B.dps_query(tree, x_c, beta, eps_v, grad=want_grad)
        else:
            n = tree.C - c_begin if n_ch is None else n_ch
            Q = x_c.shape[0]
            # rows past the device count are never written by the kernels
            f = torch.zeros((Q, n), device=x_c.device, dtype=torch.float32)
            g = torch.zeros((Q, n, 3), device=x_c.device, dtype=torch.float32) if want_grad else None
            B.dps_query_channels(tree, x_c, beta, eps_v, c_begin, n, grad=want_grad, f_out=f, g_out=g,
                                 q_count=q_count)
        # the gradients, when computed, give the backward its dL/dx directly
        # (dps_adjoint_accumulate_from_forward)
        ctx.has_g = g is not None and getattr(tree, "kernel", "dipole") == "dipole"
        ctx.save_for_backward(x_c, attrs_c, g if ctx.has_g else None)
        ctx.tree, ctx.beta, ctx.eps, ctx.opts, ctx.full = tree, float(beta), eps_v, opts, full
        ctx.n = f.shape[1]
        ctx.eps_like = eps if isinstance(eps, torch.Tensor) else None
        return f, g

    @staticmethod
    def backward(ctx, df, dg):
        x, attrs, g_fwd = ctx.saved_tensors
        tree = ctx.tree
        c_begin, n_ch, q_count, _, refit = ctx.opts
        if refit == "auto":
            _refit_if_changed(tree, attrs)
        need_attr, need_x, need_n, need_eps = ctx.needs_input_grad[:4]
        none = (None,) * 7
        if (df is None and dg is None) or not (need_attr or need_x or need_n or need_eps):
            return none
        df = None if df is None else df.contiguous().to(torch.float32)
        dn = de = None
        if need_n or need_eps:
            dg = None if dg is None else dg.contiguous().to(torch.float32)
            dx = torch.zeros((x.shape[0], 3), device=x.device, dtype=torch.float32) if need_x else None
            want = (B.WANT_NORMALS if need_n else 0) | (B.WANT_EPS if need_eps else 0)
            B.dps_adjoint_zero(tree)
            B.dps_adjoint_accumulate_ext(tree, x, ctx.beta, ctx.eps, df=df, dg=dg, want=want, c_begin=c_begin,
                                         n_channels=ctx.n, want_dx=need_x, dx_out=dx, q_count=q_count)
            dattrs, dn, de = B.dps_adjoint_finalize_ext(tree, attrs=need_attr, normals=need_n, eps=need_eps)
            if de is not None:
                de = de.to(device=ctx.eps_like.device, dtype=ctx.eps_like.dtype).reshape(ctx.eps_like.shape)
        elif dg is not None:
            if getattr(tree, "kernel", "dipole") == "monopole":
                raise RuntimeError("cotangents of the spatial gradients need the dipole kernel; a monopole-kernel "
                                   "tree differentiates its values only")
            # gradient cotangents (with the value cotangents, if any)
            dg = dg.contiguous().to(torch.float32)
            dx = torch.zeros((x.shape[0], 3), device=x.device, dtype=torch.float32) if need_x else None
            B.dps_adjoint_zero(tree)
            B.dps_adjoint_accumulate_grad(tree, x, ctx.beta, ctx.eps, dg, df=df, c_begin=c_begin, n_channels=ctx.n,
                                          want_dx=need_x, dx_out=dx, q_count=q_count)
            dattrs = B.dps_adjoint_finalize(tree)
        elif need_x and ctx.has_g:
            # dL/dx = sum_c df_c grad_c from the forward's gradients; the walk
            # accumulates the attribute derivatives only
            dx = torch.zeros((x.shape[0], 3), device=x.device, dtype=torch.float32)
            B.dps_adjoint_zero(tree)
            B.dps_adjoint_accumulate_from_forward(tree, x, ctx.beta, ctx.eps, df, g_fwd, c_begin=c_begin,
                                                  n_channels=ctx.n, dx_out=dx, q_count=q_count)
            dattrs = B.dps_adjoint_finalize(tree)
        elif ctx.full:
            dattrs, dx = B.dps_adjoint(tree, x, ctx.beta, ctx.eps, df, want_dx=need_x)
        else:
            n = df.shape[1]
            dx = torch.zeros((x.shape[0], 3), device=x.device, dtype=torch.float32) if need_x else None
            B.dps_adjoint_zero(tree)
            B.dps_adjoint_accumulate_channels(tree, x, ctx.beta, ctx.eps, c_begin, n, df, want_dx=need_x,
                                              dx_out=dx, q_count=q_count)
            dattrs = B.dps_adjoint_finalize(tree)
        dattrs = dattrs.reshape(attrs.shape) if (need_attr and dattrs is not None) else None
        return dattrs, (dx if need_x else None), dn, de, None, None, None


def dipole_sum(attrs, x, tree, beta: float, eps, *, channels=None, q_count=None, grad: bool = True,
               refit="auto", normals=None):
    """Functional form of ``DipoleSum``: returns (f, grad or None).

    channels: None (all) or (c_begin, n_channels); q_count: optional int64
    CUDA tensor [1] with the number of rows to evaluate; grad: also return the
    spatial gradients; refit: "auto" (refit when attrs changed since the last
    refit, judged from its storage and version), True (always, e.g. inside a
    captured graph) or False (never); normals: optional [M,3] tensor of point
    normals (differentiable); eps: float, or a tensor to differentiate."""
    c_begin, n_ch = (0, None) if channels is None else (int(channels[0]), int(channels[1]))
    if channels is not None and c_begin == 0 and n_ch == tree.C:
        n_ch = None
    return DipoleSum.apply(attrs, x, normals, eps, tree, beta, (c_begin, n_ch, q_count, bool(grad), refit))
