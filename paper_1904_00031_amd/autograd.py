"""log psi as a differentiable PyTorch function whose backward pass is the library's
hand-written Jacobian kernel (argument marshalling only; no arithmetic here).

For the RBM, log psi is holomorphic in the parameters with derivatives O_k (Sec. 2.2.5,
analytic RBM derivatives): O_a = s, O_b = tanh(theta), O_W = tanh(theta) s. PyTorch
passes the incoming gradient g_s = dL/dRe(log psi_s) + i dL/dIm(log psi_s) and expects
dL/dRe p_k + i dL/dIm p_k back; for a holomorphic map that is sum_s conj(O_sk) g_s,
i.e. O^dagger g, which nqs_log_psi_grad computes on the matrix cores (theta recomputed
from the spins, O never stored). Forward-mode products O v go through log_psi_jvp, and
the implicit S v of stochastic reconfiguration through sv_product.
"""
import torch


class LogPsi(torch.autograd.Function):
    """log psi(sigma) for each row of sigma; differentiable in params."""

    @staticmethod
    def forward(ctx, params, sigma, model):
        ctx.model = model
        ctx.save_for_backward(params, sigma)
        return model.log_psi(params.detach(), sigma)

    @staticmethod
    def backward(ctx, grad_out):
        params, sigma = ctx.saved_tensors
        model = ctx.model
        g = grad_out.contiguous().to(model.value_dtype)
        vjp, _ = model.log_psi_grad(params.detach(), sigma, u=g)
        return vjp.to(params.dtype), None, None


def log_psi(model, params, sigma):
    """Differentiable log psi (values double / complex double, gradient in the
    parameters' dtype)."""
    return LogPsi.apply(params, sigma, model)


def log_psi_jvp(model, params, sigma, v):
    """O v: the directional derivative of log psi along v (double / complex double)."""
    _, jvp = model.log_psi_grad(params.detach(), sigma, v=v.to(model.value_dtype).contiguous())
    return jvp


def sv_product(model, params, sigma, v, diag_shift=0.0, workspace=None):
    """(S + diag_shift I) v with S the centred covariance of O over the rows of sigma."""
    ws = model.sr_prepare(params.detach(), sigma, workspace)
    return model.sr_matvec(sigma, ws, v.to(model.value_dtype).contiguous(), diag_shift)
