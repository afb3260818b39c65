"""torch.autograd bridge: the NLL as a differentiable function of theta.

forward() runs nll_grad (one launch of the per-event adjoint kernels) and
keeps the gradient; backward() scales it by the incoming gradient.  theta
may live on any device and have any floating dtype: the library reads the
parameters on the host (as the minimiser holds them), and the value and the
gradient are returned on theta's device in theta's dtype.  The events stay
on the GPU.
"""
import numpy as np
import torch

from .core import nll_grad


class NLLFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, graph, dataset, stream=None):
        if not theta.is_floating_point():
            raise TypeError("theta must be a floating-point tensor")
        th = theta.detach().to(device="cpu", dtype=torch.float64).numpy()
        v, g = nll_grad(graph, dataset, th, stream)
        ctx.save_for_backward(torch.from_numpy(np.asarray(g, dtype=np.float64)).to(theta.device, theta.dtype))
        return torch.tensor(v, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out.to(g.device, g.dtype) * g, None, None, None


def nll(theta, graph, dataset, stream=None):
    """Differentiable NLL(theta) for a graph and an uploaded dataset."""
    return NLLFunction.apply(theta, graph, dataset, stream)
