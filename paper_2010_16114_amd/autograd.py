"""torch.autograd.Function wrappers around the hand-written adjoint.

BreslowNLL: loss_b = -L(eta_b), the negative Breslow log partial likelihood of a
linear predictor (Section 5.3).  Its derivative is -(I - P) delta = -r, which
the forward's risk-set kernel already forms (w and the reverse cumulative sums
are kept); the backward only scales it by the incoming gradient.

CoxLinearNLL: loss_b = -L(X~ beta_b); the forward computes the loss and
X~'r in one pass of the library, the backward scales the saved gradient.
"""
from __future__ import annotations

import torch


class BreslowNLL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta, cox):
        loss = cox.nll_forward(eta)
        ctx.cox = cox
        ctx.save_for_backward(eta)
        return loss.to(eta.dtype) if eta.dtype == torch.float32 else loss

    @staticmethod
    def backward(ctx, grad_loss):
        (eta,) = ctx.saved_tensors
        # the adjoint reads the state of the context's last forward; redo the
        # forward if another one ran on the same context in between
        if ctx.cox.last_forward_key != ctx.cox.forward_key(eta):
            ctx.cox.nll_forward(eta)
        grad = ctx.cox.nll_backward(grad_loss, eta)
        return grad, None


class CoxLinearNLL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta, cox):
        loss, grad = cox.loss_grad(beta, want_grad=True)
        ctx.save_for_backward(grad)
        return torch.as_tensor(loss, device=beta.device).to(beta.dtype)

    @staticmethod
    def backward(ctx, grad_loss):
        (grad,) = ctx.saved_tensors
        return grad * grad_loss.to(grad.dtype).view(-1, 1), None
