"""Pins of the oracle's COMP node (section "Combining functions":
CompositePdf, f(g(x))): with the identity core the node is its shell
normalised over the box; an exponential of a linear core is the exponential
with the product rate (a wrong chain-rule factor or argument fails); the
composition integrates to 1; the gradient matches finite differences."""
import math

import numpy as np
import pytest
from scipy import integrate

import synthgen as S

from test_oracle_pins import fd_grad


def model(oracle_mod, params, tree):
    return oracle_mod.Model({"obs": [("x", 0.0, 10.0)], "params": params, "model": tree})


def comp(core, shell):
    return {"op": "comp", "obs": "x", "children": [core, shell]}


def test_identity_core_gives_the_shell(oracle_mod):
    par = [("one", 1.0, 0.1, 0, 0, False), ("m", 6.0, 0.1, 0, 0, False), ("s", 1.3, 0.1, 0, 0, False)]
    c = model(oracle_mod, par, comp({"op": "poly", "obs": "x", "par": ["one"], "x0": 1.0},
                                    {"op": "gauss", "obs": "x", "par": ["m", "s"]}))
    g = model(oracle_mod, par, {"op": "gauss", "obs": "x", "par": ["m", "s"]})
    th = np.array([1.0, 6.0, 1.3])
    x = np.linspace(0.0, 10.0, 31)
    assert np.max(np.abs(c.logpdf(th, {"x": x}) - g.logpdf(th, {"x": x}))) < 1e-12


def test_exponential_of_a_linear_core_is_an_exponential(oracle_mod):
    par = [("a", 0.5, 0.1, 0, 0, False), ("al", -0.8, 0.1, 0, 0, False), ("r", -0.4, 0.1, 0, 0, False)]
    c = model(oracle_mod, par, comp({"op": "poly", "obs": "x", "par": ["a"], "x0": 3.0},
                                    {"op": "exp", "obs": "x", "par": ["al"]}))
    e = model(oracle_mod, par, {"op": "exp", "obs": "x", "par": ["r"]})
    th = np.array([0.5, -0.8, -0.4])
    x = np.linspace(0.0, 10.0, 23)
    assert np.max(np.abs(c.logpdf(th, {"x": x}) - e.logpdf(th, {"x": x}))) < 1e-12


def test_composition_integrates_to_one(oracle_mod):
    sp = S.workload("comp")
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    f = lambda v: math.exp(m.logpdf(th, {"x": np.array([v])}, n_threads=1)[0])
    assert abs(integrate.quad(f, 0.0, 10.0, epsabs=0, epsrel=1e-12, limit=400)[0] - 1.0) < 1e-11


def test_composition_gradient_matches_finite_differences(oracle_mod):
    sp = S.workload("comp")
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    data = {"x": np.linspace(3.0, 9.5, 40)}
    v, g = m.nll(th, data, grad=True)
    assert np.allclose(g, fd_grad(m, th, data), rtol=1e-6, atol=1e-6 * np.abs(g).max())
