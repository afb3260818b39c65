"""Pins of the oracle's DPMAP node (section "Results": in the mixing fit the
distribution of the decay-time uncertainty varies across the Dalitz plot):
a density of sigma_t conditional on the event's cell of the plot.  The
product with the time-dependent density splits into that density's NLL plus
one 1-D NLL per cell over the cell's events, with cells assigned here by
numpy's searchsorted (a transposed cell index, a boundary on the wrong side
or a missing term fails); each cell's density integrates to 1 over sigma_t."""
import copy
import math

import numpy as np
import pytest
from scipy import integrate

import synthgen as S

from helpers import gen_data, oracle_model


def _cells(data):
    b12, b13 = S.SIGMA_T_BOUNDS
    return (np.searchsorted(b12, data["s12"], side="right") * (len(b13) + 1)
            + np.searchsorted(b13, data["s13"], side="right"))


def _gauss_model(oracle_mod):
    return oracle_mod.Model({"obs": [("sigma_t", 0.02, 0.2)],
                             "params": [("m", 0.1, 0.01, 0, 0, False), ("s", 0.05, 0.01, 0, 0, False)],
                             "model": {"op": "gauss", "obs": "sigma_t", "par": ["m", "s"]}})


@pytest.fixture(scope="module")
def data():
    d = gen_data("c4s", 3000, 71)
    # events exactly on the cell boundaries (inside the plot): they belong
    # to the cell above
    d = {k: v.copy() for k, v in d.items()}
    pts = [(1.5, 1.0), (1.5, 1.2), (1.0, 1.5), (1.2, 1.5), (1.5, 1.5), (2.0, 1.5)]
    for i, (a, b) in enumerate(pts):
        d["s12"][i], d["s13"][i] = a, b
    return d


def test_product_splits_into_tddp_and_cell_nlls(oracle_mod, data):
    sp = S.workload("c4s")
    m = oracle_mod.Model(sp)
    m4 = oracle_model("c4")
    g1 = _gauss_model(oracle_mod)
    th = m.theta(sp["truth"])
    th[18:] = [0.07, 0.03, 0.11, 0.05, 0.13, 0.02, 0.09, 0.06]  # distinct cells
    v, gr = m.nll(th, data, grad=True)
    v4, g4 = m4.nll(th[:18], data, grad=True)
    cell = _cells(data)
    assert np.all(np.bincount(cell, minlength=4) > 0)
    ref, gref = v4, np.concatenate([g4, np.zeros(8)])
    for c in range(4):
        sel = cell == c
        vc, gc = g1.nll(th[18 + 2 * c:20 + 2 * c], {"sigma_t": data["sigma_t"][sel]}, grad=True)
        ref += vc
        gref[18 + 2 * c:20 + 2 * c] = gc
    assert abs(v - ref) <= 1e-12 * abs(ref)
    assert np.allclose(gr, gref, rtol=1e-11, atol=1e-9)


def test_cell_densities_integrate_to_one(oracle_mod):
    sp = copy.deepcopy(S.workload("c4s"))
    sp["model"] = sp["model"]["children"][1]
    sp["obs"] = [o for o in sp["obs"] if o[0] != "t"]
    sp["params"] = sp["params"][18:]
    sp["truth"] = {p[0]: sp["truth"][p[0]] for p in sp["params"]}
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    for s12, s13 in [(1.0, 1.0), (1.0, 2.0), (2.0, 1.0), (2.0, 2.0), (1.5, 1.5)]:
        f = lambda u: math.exp(m.logpdf(th, {"s12": np.array([s12]), "s13": np.array([s13]),
                                              "sigma_t": np.array([u])})[0])
        assert abs(integrate.quad(f, 0.02, 0.2, epsabs=0, epsrel=1e-12)[0] - 1.0) < 1e-11
