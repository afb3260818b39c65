"""Pins of the oracle's PROD over a shared observable (section "Combining
functions": ProdPdf; the product of densities on the same variable is
renormalised numerically): closed-form special cases (Gaussian x Gaussian
is a Gaussian, exponential x exponential an exponential), normalisation by
an independent quadrature, and the gradient against finite differences.
Each test names the mistake it would catch."""
import copy
import math

import numpy as np
import pytest
from scipy import integrate

import synthgen as S

from test_oracle_pins import fd_grad

OBS = [("x", 0.0, 10.0)]


def model(oracle_mod, params, tree):
    return oracle_mod.Model({"obs": OBS, "params": params, "model": tree})


def test_gauss_times_gauss_is_a_gauss(oracle_mod):
    """N(mu1, s1) N(mu2, s2) on [0, 10] = N(mu, s) with the textbook combined
    mean and width, truncated to the box (a missing renormalisation, or one
    over the wrong group, fails)."""
    par = [("m1", 4.0, 0.1, 0, 0, False), ("s1", 1.5, 0.1, 0, 0, False),
           ("m2", 6.5, 0.1, 0, 0, False), ("s2", 2.0, 0.1, 0, 0, False),
           ("m", 0.0, 0.1, 0, 0, False), ("s", 1.0, 0.1, 0, 0, False)]
    prod = model(oracle_mod, par, {"op": "prod", "children": [
        {"op": "gauss", "obs": "x", "par": ["m1", "s1"]}, {"op": "gauss", "obs": "x", "par": ["m2", "s2"]}]})
    one = model(oracle_mod, par, {"op": "gauss", "obs": "x", "par": ["m", "s"]})
    m1, s1, m2, s2 = 4.0, 1.5, 6.5, 2.0
    mu = (m1 * s2**2 + m2 * s1**2) / (s1**2 + s2**2)
    sg = math.sqrt(s1**2 * s2**2 / (s1**2 + s2**2))
    th = np.array([m1, s1, m2, s2, mu, sg])
    x = np.linspace(0.0, 10.0, 37)
    assert np.allclose(prod.logpdf(th, {"x": x}), one.logpdf(th, {"x": x}), rtol=0, atol=1e-12)


def test_exp_times_exp_is_an_exp(oracle_mod):
    par = [("a", -0.3, 0.1, 0, 0, False), ("b", 0.1, 0.1, 0, 0, False), ("c", 0.0, 0.1, 0, 0, False)]
    prod = model(oracle_mod, par, {"op": "prod", "children": [
        {"op": "exp", "obs": "x", "par": ["a"]}, {"op": "exp", "obs": "x", "par": ["b"]}]})
    one = model(oracle_mod, par, {"op": "exp", "obs": "x", "par": ["c"]})
    th = np.array([-0.3, 0.1, -0.2])
    x = np.linspace(0.0, 10.0, 23)
    assert np.allclose(prod.logpdf(th, {"x": x}), one.logpdf(th, {"x": x}), rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", ["shared", "shared_sum"])
def test_shared_product_normalised(oracle_mod, name):
    sp = S.workload(name)
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    f = lambda x: math.exp(m.logpdf(th, {"x": np.array([x])})[0])
    tot = integrate.quad(f, 0.0, 10.0, epsabs=0, epsrel=1e-12, limit=400)[0]
    assert abs(tot - 1.0) < 1e-11


def test_shared_product_times_independent_y_normalised(oracle_mod):
    """The shared group on x is renormalised on its own; the exponential in y
    keeps its closed-form normalisation (a renormalisation over both fails)."""
    sp = S.workload("shared_2d")
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    f = lambda y, x: math.exp(m.logpdf(th, {"x": np.array([x]), "y": np.array([y])})[0])
    tot = integrate.dblquad(f, 0.0, 10.0, 0.0, 5.0, epsabs=0, epsrel=1e-11)[0]
    assert abs(tot - 1.0) < 1e-9


@pytest.mark.parametrize("name", ["shared", "shared_sum", "shared_2d"])
def test_shared_product_gradient_matches_finite_differences(oracle_mod, name):
    sp = S.workload(name)
    m = oracle_mod.Model(sp)
    rng = np.random.default_rng(6)
    th = m.theta(sp["truth"]) * (1 + 0.05 * rng.standard_normal(len(sp["params"])))
    d = {"x": rng.uniform(0.0, 10.0, 400)}
    if name == "shared_2d":
        d["y"] = rng.uniform(0.0, 5.0, 400)
    v, g = m.nll(th, d, grad=True)
    gf = fd_grad(m, th, d, rel=1e-6)
    scale = np.abs(m.logpdf(th, d, grad_rows=True)[1]).sum(axis=0)
    assert np.all(np.abs(g - gf) <= 1e-7 * scale + 1e-7)
