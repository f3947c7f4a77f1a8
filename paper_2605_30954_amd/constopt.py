"""Constant optimisation driven by the fitness gradient: Adam steps (Kingma &
Ba 2015) on every program's constants, each step one fused fitness + gradient
call (gpgomea_grad_consts) followed by the library's Adam kernel
(gpgomea_adam_consts).  The paper names real-valued constant optimisation as
the next thing to integrate with GPU evaluation (Section 5)."""
import ctypes
import math

from . import _dev_tensor, _stream, _torch, check, eval_batch, grad_consts, lib

__all__ = ["adam_step", "optimise_constants"]


def adam_step(consts, grad, fitness, moments, best_consts, best_fitness, t, lr, beta1=0.9,
              beta2=0.999, eps=1e-12):
    """gpgomea_adam_consts on device tensors: consts float32 [M, C] (in place),
    grad float64 [M, C], fitness float64 [M], moments float32 [2, M, C],
    best_consts float32 [M, C], best_fitness float64 [M] (both in place)."""
    torch = _torch()
    consts = _dev_tensor(consts, torch.float32, "consts")
    dev = consts.device
    M, C = consts.shape
    grad = _dev_tensor(grad, torch.float64, "grad", dev)
    fitness = _dev_tensor(fitness, torch.float64, "fitness", dev)
    moments = _dev_tensor(moments, torch.float32, "moments", dev)
    best_consts = _dev_tensor(best_consts, torch.float32, "best_consts", dev)
    best_fitness = _dev_tensor(best_fitness, torch.float64, "best_fitness", dev)
    if grad.shape != (M, C) or moments.shape != (2, M, C) or best_consts.shape != (M, C) or \
            fitness.shape != (M,) or best_fitness.shape != (M,):
        raise ValueError("expected consts/grad/best_consts [M, C], moments [2, M, C], fitness [M]")
    check(lib.gpgomea_adam_consts(
        consts.data_ptr(), M, C, grad.data_ptr(), fitness.data_ptr(), moments.data_ptr(),
        best_consts.data_ptr(), best_fitness.data_ptr(), int(t), float(lr), float(beta1),
        float(beta2), float(eps), ctypes.c_void_p(_stream(dev).cuda_stream)))


def optimise_constants(ops, consts, X, y, steps=100, lr=0.02, beta1=0.9, beta2=0.999, eps=1e-12,
                       linear_scaling=True):
    """Run ``steps`` Adam steps on the constants of every program; return
    (best constants float32 [M, C], their fitness float64 [M]).  The start
    point counts: no program ends worse than it began."""
    torch = _torch()
    if not isinstance(consts, torch.Tensor) or not consts.is_cuda:
        raise ValueError("consts must be a GPU tensor (this library has no CPU path)")
    M, C = consts.shape
    dev = consts.device
    cs = consts.detach().clone().contiguous()
    best_c = cs.clone()
    best_f = torch.full((M,), math.inf, dtype=torch.float64, device=dev)
    moments = torch.zeros((2, M, C), dtype=torch.float32, device=dev)
    grad = None
    for t in range(1, int(steps) + 1):
        fit, grad = grad_consts(ops, cs, X, y, linear_scaling=linear_scaling)
        adam_step(cs, grad, fit, moments, best_c, best_f, t, lr, beta1, beta2, eps)
    # the point the last step reached: record it if it is the best (lr = 0)
    fit = eval_batch(ops, cs, X, y, linear_scaling=linear_scaling)
    if grad is None:
        grad = torch.zeros((M, C), dtype=torch.float64, device=dev)
    adam_step(cs, grad, fit, moments, best_c, best_f, int(steps) + 1, 0.0, beta1, beta2, eps)
    return best_c, best_f
