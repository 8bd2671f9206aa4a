"""S_f(U) as a torch.autograd.Function whose backward is the HIP force kernel.

Forward: X^(j) = (A[U] + beta_j)^-1 phi for all poles (bms_solve), then
  S_f = sum_i phi_i^dag (a0 phi_i + sum_j alpha_j X^(j)_i)        (Sec. II, eq. RA)
Backward: dS_f/dU from bms_force (eq. force), returned in PyTorch's complex
convention (dL/dRe U + i dL/dIm U), times the incoming real gradient.
The gauge field U is the only differentiable input.
"""
import torch

from . import bms


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, U, phi, ctx, mass, a0, alpha, beta, tol, max_iter):
        ctx.set_gauge(U.detach().contiguous())
        X, st = ctx.solve(mass, list(beta), phi.detach().contiguous(), tol=tol, max_iter=max_iter)
        S = ctx.action(a0, list(alpha), phi.detach().contiguous(), X)
        fctx.save_for_backward(X)
        fctx.bctx = ctx
        fctx.alpha = list(alpha)
        fctx.gauge = U.detach().contiguous()
        fctx.stats = st
        return torch.tensor(sum(S), dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(fctx, grad_out):
        (X,) = fctx.saved_tensors
        ctx = fctx.bctx
        ctx.set_gauge(fctx.gauge)  # the context may have been reused since forward
        G = ctx.force(fctx.alpha, X, bms.BMS_FORCE_RAW)
        return (grad_out.to(G.dtype) * G, None, None, None, None, None, None, None, None)


def pseudofermion_action(U, phi, ctx, mass, rational, tol=1e-10, max_iter=20000):
    """S_f(U) for pseudofermions phi[cb][3][n] and a rational approximation
    r(x) = a0 + sum alpha_j / (x + beta_j) (an inputs.RationalApprox)."""
    return PseudofermionAction.apply(U, phi, ctx, mass, rational.a0, rational.alpha.tolist(),
                                     rational.beta.tolist(), tol, max_iter)
