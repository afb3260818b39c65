"""hipfit: unbinned maximum-likelihood fits on MI355X (gfx950).

The per-event PDF-tree evaluation, the adjoint gradient, the reductions, the
normalisation grids and the minimiser run in libhipfit.so (hand-written HIP
kernels + C++ runtime, C ABI in include/hipfit.h).  This package binds that
library; PyTorch is used only for device streams (and the autograd wrapper).
"""
from ._lib import HipfitError, lib  # noqa: F401
from .core import (FP32_EVAL, FP64, Dataset, Graph, fit, nll_eval, nll_grad,  # noqa: F401
                   minimize, nll_grad_batched, nll_grad_noalloc, nll_terms, profile,
                   version)
from .serving import BatchEngine, FitServer, serve_one_at_a_time  # noqa: F401,E402


def autograd_nll(theta, graph, dataset, stream=None):
    """Differentiable NLL (torch.autograd) -- see paper_1311_1753_amd.autograd."""
    from .autograd import nll
    return nll(theta, graph, dataset, stream)
from .pdfs import (AddPdf, DalitzPdf, ExpPdf, FitManager, GaussianPdf, GooPdf,  # noqa: F401,E402
                   PolynomialPdf, ProdPdf, TddpPdf, UnbinnedDataSet, Variable)
