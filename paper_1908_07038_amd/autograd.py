"""torch.autograd wrappers whose backward passes are the hand-written adjoint
kernels (gradient, divergence and curl adjoints).

The adjoints are exact transposes for the plain Euclidean inner product, so
for a loss l(grad f) the input gradient is gradient_adjoint(dl/dgrad); the
Laplacian L = D G has the adjoint G^T D^T.
"""

import torch

from . import (curl, curl_adjoint, divergence, divergence_adjoint, divergence_curl, divergence_gradient_adjoint,
               gradient, gradient_adjoint, gradient_laplacian, laplacian)


class Gradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mesh, f):
        ctx.mesh = mesh
        return gradient(mesh, f.contiguous())

    @staticmethod
    def backward(ctx, gbar):
        return None, gradient_adjoint(ctx.mesh, gbar.contiguous())


class Divergence(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mesh, uv):
        ctx.mesh = mesh
        return divergence(mesh, uv.contiguous())

    @staticmethod
    def backward(ctx, dbar):
        return None, divergence_adjoint(ctx.mesh, dbar.contiguous())


class Laplacian(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mesh, f):
        ctx.mesh = mesh
        return laplacian(mesh, f.contiguous())

    @staticmethod
    def backward(ctx, lbar):
        return None, gradient_adjoint(ctx.mesh, divergence_adjoint(ctx.mesh, lbar.contiguous()))


class Curl(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mesh, uv):
        ctx.mesh = mesh
        return curl(mesh, uv.contiguous())

    @staticmethod
    def backward(ctx, zbar):
        return None, curl_adjoint(ctx.mesh, zbar.contiguous())


class GradientLaplacian(torch.autograd.Function):
    """(grad f, lap f) in one pass; backward G^T (gbar + D^T lbar)."""

    @staticmethod
    def forward(ctx, mesh, f):
        ctx.mesh = mesh
        return gradient_laplacian(mesh, f.contiguous())

    @staticmethod
    def backward(ctx, gbar, lbar):
        w = gbar.contiguous() if gbar is not None else None
        if lbar is not None:
            t = divergence_adjoint(ctx.mesh, lbar.contiguous())
            w = t if w is None else w + t
        return None, gradient_adjoint(ctx.mesh, w)


class DivergenceCurl(torch.autograd.Function):
    """(div uv, curl uv) in one pass; backward D^T dbar + C^T zbar."""

    @staticmethod
    def forward(ctx, mesh, uv):
        ctx.mesh = mesh
        return divergence_curl(mesh, uv.contiguous())

    @staticmethod
    def backward(ctx, dbar, zbar):
        out = None
        if dbar is not None:
            out = divergence_adjoint(ctx.mesh, dbar.contiguous())
        if zbar is not None:
            t = curl_adjoint(ctx.mesh, zbar.contiguous())
            out = t if out is None else out + t
        return None, out


class DivergenceGradientAdjoint(torch.autograd.Function):
    """(div uv, G^T uv) in one pass; backward D^T dbar + G fbar_bar (the
    gradient is the adjoint of the gradient adjoint)."""

    @staticmethod
    def forward(ctx, mesh, uv):
        ctx.mesh = mesh
        return divergence_gradient_adjoint(mesh, uv.contiguous())

    @staticmethod
    def backward(ctx, dbar, fbar):
        out = None
        if dbar is not None:
            out = divergence_adjoint(ctx.mesh, dbar.contiguous())
        if fbar is not None:
            t = gradient(ctx.mesh, fbar.contiguous())
            out = t if out is None else out + t
        return None, out


class RemapFunction(torch.autograd.Function):
    """Remap of a node field (see Remap); backward the exact transpose."""

    @staticmethod
    def forward(ctx, r, f):
        ctx.r = r
        return r(f.contiguous())

    @staticmethod
    def backward(ctx, ybar):
        return None, ctx.r.adjoint(ybar.contiguous())


def grad(mesh, f):
    return Gradient.apply(mesh, f)


def div(mesh, uv):
    return Divergence.apply(mesh, uv)


def lap(mesh, f):
    return Laplacian.apply(mesh, f)


def rot(mesh, uv):
    """Differentiable curl (vertical vorticity)."""
    return Curl.apply(mesh, uv)


def grad_lap(mesh, f):
    """Differentiable (gradient, Laplacian) of one field in one pass."""
    return GradientLaplacian.apply(mesh, f)


def div_rot(mesh, uv):
    """Differentiable (divergence, curl) of one vector field in one pass."""
    return DivergenceCurl.apply(mesh, uv)


def div_gradt(mesh, uv):
    """Differentiable (divergence, gradient adjoint) of one vector field in one pass."""
    return DivergenceGradientAdjoint.apply(mesh, uv)


def remap(r, f):
    """Differentiable remap of f [V][L] with the Remap r."""
    return RemapFunction.apply(r, f)

