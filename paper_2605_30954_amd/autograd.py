"""torch.autograd face of the constant gradient.

    f = GPGOMEAFitness.apply(consts, ops, X, y)    # float64 [M]
    f.sum().backward()                            # consts.grad = d f_i / d consts[i]

The forward pass runs gpgomea_grad_consts (fitness and gradient in one
call); backward scales the saved gradient by grad_output.  Gradients flow to
the constants only.
"""
import torch


class GPGOMEAFitness(torch.autograd.Function):
    @staticmethod
    def forward(ctx, consts, ops, X, y, linear_scaling=True):
        from . import grad_consts
        fit, grad = grad_consts(ops, consts.detach(), X, y, linear_scaling=linear_scaling)
        ctx.save_for_backward(grad)
        ctx.cdtype = consts.dtype
        return fit

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        g = (grad_out.to(grad.dtype)[:, None] * grad).to(ctx.cdtype)
        return g, None, None, None, None
