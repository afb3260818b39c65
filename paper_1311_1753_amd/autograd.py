"""torch.autograd bridge: the NLL as a differentiable function of theta.

forward() runs nll_grad (one launch of the per-event adjoint kernels) and
keeps the gradient; backward() scales it by the incoming gradient.  theta is
a float64 CPU tensor (the parameters live on the host, as in the minimiser);
the events stay on the GPU.
"""
import numpy as np
import torch

from .core import nll_grad


class NLLFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, graph, dataset, stream=None):
        th = theta.detach().to(torch.float64).cpu().numpy()
        v, g = nll_grad(graph, dataset, th, stream)
        ctx.save_for_backward(torch.from_numpy(np.asarray(g, dtype=np.float64)))
        return torch.tensor(v, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None


def nll(theta, graph, dataset, stream=None):
    """Differentiable NLL(theta) for a graph and an uploaded dataset."""
    return NLLFunction.apply(theta, graph, dataset, stream)
