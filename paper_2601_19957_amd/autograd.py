"""Differentiable log-likelihood on the GPU: forward, backward and double backward
run in the library's hand-written kernels (sb_logl_grad_dev, sb_hvp_dev).

``logl(model, X)`` returns l(X) for the rows of X.  Its backward is the
analytic gradient kernel; the gradient is itself a differentiable function
whose backward is the Hessian-vector-product kernel (the Hessian is
symmetric, so the vector-Jacobian product of grad l is H v).  Hence
``torch.autograd.grad`` with ``create_graph=True`` and
``torch.autograd.functional.hvp`` work on device tensors, and exact Hessians
replace the finite-difference stencils of the paper's appendix
("Gradient and Hessian Computation").
"""
from __future__ import annotations

import torch

from . import _lib


class LogLHvp(torch.autograd.Function):
    """HV = H(X) V per row (FP64 kernel).  Linear in V with a symmetric H, so
    the vector-Jacobian product in V is H(X) applied to the incoming vector;
    third derivatives in X are not provided."""

    @staticmethod
    def forward(ctx, X, V, model):
        hv = _lib.sb_hvp_dev(model, X.detach().to(torch.float64), V.detach().to(torch.float64))
        ctx.save_for_backward(X)
        ctx.model = model
        return hv.to(V.dtype)

    @staticmethod
    def backward(ctx, gH):
        (X,) = ctx.saved_tensors
        return None, LogLHvp.apply(X, gH, ctx.model), None


class LogLGrad(torch.autograd.Function):
    """G = grad l(X), row-wise; backward gives H(X) gG per row."""

    @staticmethod
    def forward(ctx, X, model):
        _, G = _lib.sb_logl_grad_dev(model, X)
        ctx.save_for_backward(X)
        ctx.model = model
        return G

    @staticmethod
    def backward(ctx, gG):
        (X,) = ctx.saved_tensors
        return LogLHvp.apply(X, gG, ctx.model).to(X.dtype), None


class LogL(torch.autograd.Function):
    """l(X) for the rows of X (float64: FP64 path; float32: FP32 path)."""

    @staticmethod
    def forward(ctx, X, model):
        l = _lib.sb_logl_grad_dev(model, X, grad=False)
        ctx.save_for_backward(X)
        ctx.model = model
        return l

    @staticmethod
    def backward(ctx, gl):
        (X,) = ctx.saved_tensors
        G = LogLGrad.apply(X, ctx.model)
        return gl[:, None] * G, None


def logl(model, X):
    """Differentiable l at the rows of X; ``model`` is a ``_lib.DeviceModel``."""
    return LogL.apply(X, model)


class UserLogL(torch.autograd.Function):
    """l(X) of a run-time compiled user likelihood (``_lib.UserLogL``), FP64; its backward is
    the central finite-difference gradient of the same batch kernels (step ``eps``), the
    derivative a likelihood without an analytic backward has (appendix "Gradient and Hessian
    Computation").  Second derivatives are not provided here (``UserLogL.fd(full=True)`` gives
    the FD Hessian)."""

    @staticmethod
    def forward(ctx, X, fn, params, eps):
        X64 = X.detach().to(torch.float64)
        l = fn.logl(X64, params)
        ctx.save_for_backward(X64)
        ctx.fn, ctx.params, ctx.eps = fn, params, eps
        return l.to(X.dtype)

    @staticmethod
    def backward(ctx, gl):
        (X,) = ctx.saved_tensors
        G = ctx.fn.fd(X, ctx.eps, ctx.params)["grad"]
        return (gl.to(torch.float64)[:, None] * G).to(gl.dtype), None, None, None


def user_logl(fn, X, params=None, eps: float = 1e-5):
    """Differentiable l of a user likelihood at the rows of X (FD gradient on backward)."""
    return UserLogL.apply(X, fn, params, eps)
