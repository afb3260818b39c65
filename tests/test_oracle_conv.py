"""Pins of the oracle's CONV node (section "Combining functions":
ConvolutionPdf, here a sum over a grid of the model's box): a Gaussian model
smeared by a Gaussian resolution is the Gaussian of the summed variances; an
exponential model smeared by a Gaussian approaches the closed form of the
convolution integral with the midpoint rule's 1/N^2 error; each density
integrates to 1 (a wrong Z, a residual range applied on the wrong side or a
dropped grid term fails); the gradient matches finite differences."""
import copy
import math

import numpy as np
import pytest
from scipy import integrate, special

import synthgen as S

from test_oracle_pins import fd_grad


def model(oracle_mod, params, tree, box=(0.0, 10.0)):
    return oracle_mod.Model({"obs": [("x",) + tuple(box)], "params": params, "model": tree})


def conv(grid, d_lo, d_hi, m, r):
    return {"op": "conv", "obs": "x", "grid": grid, "d_lo": d_lo, "d_hi": d_hi, "children": [m, r]}


def test_gauss_smeared_by_gauss_is_a_gauss(oracle_mod):
    par = [("m", 5.0, 0.1, 0, 0, False), ("s", 0.6, 0.1, 0, 0, False), ("rm", 0.1, 0.1, 0, 0, False),
           ("rs", 0.3, 0.1, 0, 0, False)]
    c = model(oracle_mod, par, conv(2000, -3.0, 3.0, {"op": "gauss", "obs": "x", "par": ["m", "s"]},
                                     {"op": "gauss", "obs": "x", "par": ["rm", "rs"]}))
    th = np.array([5.0, 0.6, 0.1, 0.3])
    x = np.linspace(3.0, 7.2, 29)
    sg = math.sqrt(0.6 ** 2 + 0.3 ** 2)
    ref = -0.5 * ((x - 5.1) / sg) ** 2 - math.log(sg * math.sqrt(2 * math.pi))
    assert np.max(np.abs(c.logpdf(th, {"x": x}) - ref)) < 1e-9


def _exp_gauss(x, al, rm, rs, lo, hi):
    """ln of int_lo^hi e^{al t} N(x - t; rm, rs) dt (closed form)."""
    mu = x - rm + al * rs ** 2  # completing the square in t
    return (al * (x - rm) + 0.5 * al ** 2 * rs ** 2
            + np.log(0.5 * (special.erf((hi - mu) / (math.sqrt(2) * rs)) - special.erf((lo - mu) / (math.sqrt(2) * rs)))))


def test_exp_smeared_by_gauss_converges_to_the_integral(oracle_mod):
    par = [("a", -0.4, 0.1, 0, 0, False), ("rm", 0.05, 0.1, 0, 0, False), ("rs", 0.3, 0.1, 0, 0, False)]
    th = np.array([-0.4, 0.05, 0.3])
    x = np.linspace(0.3, 9.7, 17)
    ref = _exp_gauss(x, -0.4, 0.05, 0.3, 0.0, 10.0)
    ref = ref - ref[0]
    err = []
    for n in (1000, 2000):
        c = model(oracle_mod, par, conv(n, -4.0, 4.0, {"op": "exp", "obs": "x", "par": ["a"]},
                                         {"op": "gauss", "obs": "x", "par": ["rm", "rs"]}))
        lp = c.logpdf(th, {"x": x})
        err.append(np.max(np.abs((lp - lp[0]) - ref)))
    assert err[1] < 5e-6
    assert 3.5 < err[0] / err[1] < 4.5  # midpoint rule: error ~ 1/N^2


@pytest.mark.parametrize("name", ["conv", "conv_poly"])
def test_convolutions_integrate_to_one(oracle_mod, name):
    sp = S.workload(name)
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    f = lambda v: math.exp(m.logpdf(th, {"x": np.array([v])})[0])
    # the integrand has kinks where the residual range starts or ends at a
    # grid point; quad over many pieces
    edges = np.linspace(0.0, 10.0, 81)
    tot = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11, limit=200)[0] for a, b in zip(edges[:-1], edges[1:]))
    assert abs(tot - 1.0) < 1e-8


@pytest.mark.parametrize("name", ["conv", "conv_poly"])
def test_convolution_gradient_matches_finite_differences(oracle_mod, name):
    sp = S.workload(name)
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    x = np.linspace(0.5, 9.5, 40)
    data = {"x": x}
    v, g = m.nll(th, data, grad=True)
    fd = fd_grad(m, th, data)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-6 * np.abs(g).max())
