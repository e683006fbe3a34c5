"""Differentiable operators.

The measurement operator R (degridding) is R-linear from real images to
complex visibilities (Sect. 2, eq. 3 and the remark that R maps a real to a
complex vector space).  For a real loss L, PyTorch hands the backward pass
g = dL/dRe(d) + i dL/dIm(d); the gradient with respect to the real image is
then Re(R^H g), which is exactly the gridder (the adjoint with the real part
taken, Sect. 5).  Conversely the gridder's backward is the degridder.  Both
directions run in the HIP kernels of the plan.
"""
import torch


class Degrid(torch.autograd.Function):
    """vis = wgt * R(image); backward: grad_image = Re R^H (wgt * grad_vis)."""

    @staticmethod
    def forward(ctx, image, plan, wgt=None):
        ctx.plan = plan
        ctx.has_wgt = wgt is not None
        if wgt is not None:
            ctx.save_for_backward(wgt)
        return plan.degrid(image.contiguous(), wgt=wgt)

    @staticmethod
    def backward(ctx, grad_vis):
        wgt = ctx.saved_tensors[0] if ctx.has_wgt else None
        grad_image = None
        if ctx.needs_input_grad[0]:
            grad_image = ctx.plan.grid(grad_vis.contiguous(), wgt=wgt)
        return grad_image, None, None


class Grid(torch.autograd.Function):
    """image = Re R^H (wgt * vis); backward: grad_vis = wgt * R(grad_image)."""

    @staticmethod
    def forward(ctx, vis, plan, wgt=None):
        ctx.plan = plan
        ctx.has_wgt = wgt is not None
        if wgt is not None:
            ctx.save_for_backward(wgt)
        return plan.grid(vis.contiguous(), wgt=wgt)

    @staticmethod
    def backward(ctx, grad_image):
        wgt = ctx.saved_tensors[0] if ctx.has_wgt else None
        grad_vis = None
        if ctx.needs_input_grad[0]:
            grad_vis = ctx.plan.degrid(grad_image.contiguous(), wgt=wgt)
        return grad_vis, None, None


def degrid(image, plan, wgt=None):
    return Degrid.apply(image, plan, wgt)


def grid(vis, plan, wgt=None):
    return Grid.apply(vis, plan, wgt)


def lipschitz_estimate(plan, iters=10, seed=0):
    """Largest eigenvalue of R^H R by power iteration (step size for gradient
    descent on 0.5 ||R x - d||^2)."""
    gen = torch.Generator(device=plan.device).manual_seed(seed)
    x = torch.randn((plan.npix_x, plan.npix_y), dtype=plan.real_dtype, device=plan.device, generator=gen)
    lam = 0.0
    for _ in range(iters):
        x = x / torch.linalg.vector_norm(x)
        y = plan.grid(plan.degrid(x))
        lam = float(torch.sum(x * y))
        x = y
    return lam


def gradient_descent(plan, data, steps, step_size, x0=None, wgt=None):
    """Minimise 0.5 ||wgt R x - data||^2 over real images x with plain
    gradient descent, the gradient coming from autograd through Degrid."""
    x = torch.zeros((plan.npix_x, plan.npix_y), dtype=plan.real_dtype, device=plan.device) if x0 is None \
        else x0.clone()
    losses = []
    for _ in range(steps):
        x.requires_grad_(True)
        r = degrid(x, plan, wgt) - data
        loss = 0.5 * torch.sum(r.real ** 2 + r.imag ** 2)
        (g,) = torch.autograd.grad(loss, x)
        losses.append(loss.detach())
        x = (x.detach() - step_size * g)
    return x.detach(), [float(v) for v in losses]
