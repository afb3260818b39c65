"""torch.autograd bridge and the paper-shaped API on the GPU."""
import numpy as np
import pytest

import synthgen as S
from helpers import get_spec, oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1311_1753_amd as P
    return P


def test_autograd_gradcheck(P):
    import torch
    g = P.Graph.from_spec(get_spec("c2"))
    ds = P.Dataset(g, S.gen_c2(n=20_000, seed=4), "fp64")
    th = torch.tensor([0.31, 5.2801, 0.0031, -2.1], dtype=torch.float64, requires_grad=True)
    v = P.autograd_nll(th, g, ds)
    v.backward()
    ref_v, ref_g = P.nll_grad(g, ds, th.detach().numpy())
    assert v.item() == ref_v and np.array_equal(th.grad.numpy(), ref_g)
    # gradient against central differences of the forward
    f = lambda t: P.autograd_nll(t, g, ds)
    assert torch.autograd.gradcheck(f, (th,), eps=1e-7, atol=1e-4, rtol=1e-5)


def test_autograd_with_theta_on_the_gpu(P):
    """theta as a CUDA tensor: value and gradient come back on its device,
    equal to the host-theta results."""
    import torch
    g = P.Graph.from_spec(get_spec("c2"))
    ds = P.Dataset(g, S.gen_c2(n=20_000, seed=4), "fp64")
    th = torch.tensor([0.31, 5.2801, 0.0031, -2.1], dtype=torch.float64, device="cuda", requires_grad=True)
    v = P.autograd_nll(th, g, ds)
    assert v.device == th.device
    (2.0 * v).backward()
    assert th.grad.device == th.device
    ref_v, ref_g = P.nll_grad(g, ds, th.detach().cpu().numpy())
    assert v.item() == ref_v and np.array_equal(th.grad.cpu().numpy(), 2.0 * ref_g)


def test_listing1_flow_matches_oracle(P):
    """Variables -> UnbinnedDataSet.addEvent -> ExpPdf.setData -> FitManager.fit."""
    xvar = P.Variable("xvar", 0.0, 10.0)
    alpha = P.Variable("alpha", -2.0, 0.1, -10.0, 10.0)
    data = P.UnbinnedDataSet(xvar)
    for v in S.gen_c1(n=20_000, seed=31)["x"]:
        xvar.value = v
        data.addEvent()
    pdf = P.ExpPdf("exppdf", xvar, alpha)
    pdf.setData(data)
    P.FitManager(pdf).fit()
    ref = oracle_for("c1").fit({"x": data.columns()["xvar"]})
    assert abs(alpha.value - ref["theta"][0]) <= 1e-3 * ref["errors"][0]
    assert abs(alpha.error / ref["errors"][0] - 1) < 1e-3


def test_listing2_product_fit(P):
    x = P.Variable("x", 0.0, 10.0)
    y = P.Variable("y", 0.0, 10.0)
    ax = P.Variable("alpha_x", -2.4, 0.1, -10, 10)
    ay = P.Variable("alpha_y", -1.1, 0.1, -10, 10)
    prod = P.ProdPdf("product", [P.ExpPdf("exp_x", x, ax), P.ExpPdf("exp_y", y, ay)])
    d = S.gen_listing2(n=50_000, seed=8)
    prod.setData(d, "fp32")
    r = P.FitManager(prod).fit()
    ref = oracle_for("listing2").fit(d)
    assert r["status"] == "OK"
    assert np.max(np.abs(r["theta"] - ref["theta"]) / ref["errors"]) <= 1e-3
