"""torch.autograd wrappers whose backward passes are the hand-written adjoint
kernels (gradient, divergence and curl adjoints).

The adjoints are exact transposes for the plain Euclidean inner product, so
for a loss l(grad f) the input gradient is gradient_adjoint(dl/dgrad); the
Laplacian L = D G has the adjoint G^T D^T.
"""

import torch

from . import curl, curl_adjoint, divergence, divergence_adjoint, gradient, gradient_adjoint, laplacian


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


def grad(mesh, f):
    return Gradient.apply(mesh, f)


def div(mesh, uv):
    return Divergence.apply(mesh, uv)


def lap(mesh, f):
    return Laplacian.apply(mesh, f)


def rot(mesh, uv):
    """Differentiable curl (vertical vorticity)."""
    return Curl.apply(mesh, uv)
