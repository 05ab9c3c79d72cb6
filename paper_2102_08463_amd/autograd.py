"""Differentiable 1D / 2D / 3D type 1 / type 2 transforms (torch.autograd.Function).

Backward passes run in the library:
  type 2, c = A(x) f:  grad_f = A^H g       (adjoint execute: type 1, sign -s)
                       grad_x = Re(conj(g) dc/dx)   (ES-derivative interpolation)
  type 1, f = A(x) c:  grad_c = A^H g       (adjoint execute: type 2, sign -s)
                       grad_x = Re(conj(c) d/dx [type 2, sign -s, of g])
with complex gradients in torch's convention g = dL/dRe + i dL/dIm.
The plan (and its bin-sort) is made in forward and reused by backward; it
lives as long as the autograd graph holds the context (backward may run more
than once with retain_graph) and is freed with it.
"""
import torch

from .plan import Plan


def _points(ctx_pts, dim):
    return [p.detach().contiguous() for p in ctx_pts[:dim]]


class _Type2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, eps, isign, method, x, y, z):
        dim = 1 if y is None else (2 if z is None else 3)
        n_modes = tuple(f.shape[-dim:][::-1])
        T = f.shape[0] if f.ndim == dim + 1 else 1
        plan = Plan(2, n_modes, T, eps, isign, dtype=f.dtype, method=method, device=f.device)
        pts = [p.detach() for p in (x, y, z)[:dim]]
        plan.setpts(*[p.contiguous() for p in pts])
        fc = f.detach().contiguous()
        c = plan.execute(fc)
        ctx.plan = plan
        ctx.dim = dim
        ctx.save_for_backward(fc)
        return c

    @staticmethod
    def backward(ctx, gc):
        (fc,) = ctx.saved_tensors
        plan = ctx.plan
        gc = gc.contiguous()
        gf = plan.execute_adjoint(gc).reshape(fc.shape) if ctx.needs_input_grad[0] else None
        gx = gy = gz = None
        if any(ctx.needs_input_grad[4:4 + ctx.dim]):
            gr = list(plan.interp_grad(fc, gc)) + [None] * (3 - ctx.dim)
            gx, gy, gz = gr
        return gf, None, None, None, gx, gy, gz


class _Type1(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, n_modes, eps, isign, method, x, y, z):
        dim = len(n_modes)
        T = c.shape[0] if c.ndim == 2 else 1
        plan = Plan(1, n_modes, T, eps, isign, dtype=c.dtype, method=method, device=c.device)
        pts = [p.detach() for p in (x, y, z)[:dim]]
        plan.setpts(*[p.contiguous() for p in pts])
        cc = c.detach().contiguous()
        f = plan.execute(cc)
        ctx.plan = plan
        ctx.dim = dim
        ctx.save_for_backward(cc)
        return f

    @staticmethod
    def backward(ctx, gf):
        (cc,) = ctx.saved_tensors
        plan = ctx.plan
        gf = gf.contiguous()
        gc = plan.execute_adjoint(gf).reshape(cc.shape) if ctx.needs_input_grad[0] else None
        gx = gy = gz = None
        if any(ctx.needs_input_grad[5:5 + ctx.dim]):
            gr = list(plan.interp_grad(gf, cc)) + [None] * (3 - ctx.dim)
            gx, gy, gz = gr
        return gc, None, None, None, None, gx, gy, gz


def nufft_type2(points, f, eps=1e-6, isign=+1, method="auto"):
    """Differentiable type 2: c_j = sum_k f_k exp(isign i k.x_j), w.r.t. f and the points
    (points = (x,), (x, y) or (x, y, z))."""
    p = list(points) + [None] * (3 - len(points))
    return _Type2.apply(f, eps, isign, method, p[0], p[1], p[2])


def nufft_type1(points, c, n_modes, eps=1e-6, isign=-1, method="auto"):
    """Differentiable type 1: f_k = sum_j c_j exp(isign i k.x_j), w.r.t. c and the points."""
    p = list(points) + [None] * (3 - len(points))
    return _Type1.apply(c, tuple(int(n) for n in n_modes), eps, isign, method, p[0], p[1], p[2])
