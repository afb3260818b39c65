"""Pins of the oracle's MAP node (the MappedPdf of section "Combining
functions": a different density on each range of x): normalisation over the
box by quadrature, the value at points against the separately evaluated
children and a quadrature of Z, the reduction to a single child, and the
gradient against finite differences.  Each test names the mistake it would
catch."""
import copy
import math

import numpy as np
import pytest
from scipy import integrate

import synthgen as S

from test_oracle_pins import fd_grad

BOUNDS = S.MAPPED["model"]["bounds"]


def density(m, th, x):
    return np.exp(m.logpdf(th, {"x": np.atleast_1d(np.asarray(x, dtype=float))}))


def single_child_spec(j):
    sp = copy.deepcopy(S.MAPPED)
    sp["model"] = copy.deepcopy(S.MAPPED["model"]["children"][j])
    return sp


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_map_normalised_over_the_box(oracle_mod, perturb):
    """int P dx = 1 (a Z built from the wrong ranges or from unnormalised
    children fails)."""
    m = oracle_mod.Model(S.MAPPED)
    th = m.theta(S.MAPPED["truth"]) * (1 + perturb * np.array([1, -0.2, 0.5, -1, 0.7]))
    tot = integrate.quad(lambda x: density(m, th, x)[0], 0.0, 10.0, points=BOUNDS, epsabs=0, epsrel=1e-12,
                         limit=400)[0]
    assert abs(tot - 1.0) < 1e-11


def test_map_value_is_the_selected_child_over_z(oracle_mod):
    """P(x) = P_j(x) / Z with P_j the child alone (normalised over the box) and
    Z the quadrature of the piecewise children (a wrong child selection at
    or near a boundary, or a wrong Z, fails)."""
    m = oracle_mod.Model(S.MAPPED)
    th = m.theta(S.MAPPED["truth"])
    kids = [oracle_mod.Model(single_child_spec(j)) for j in range(3)]
    names = [p[0] for p in S.MAPPED["params"]]

    def child_p(j, x):
        k = kids[j]
        return density(k, k.theta({n: th[names.index(n)] for n in k.par_names}), x)[0]

    edges = [0.0] + BOUNDS + [10.0]
    Z = sum(integrate.quad(lambda x, j=j: child_p(j, x), edges[j], edges[j + 1], epsabs=0, epsrel=1e-13)[0]
            for j in range(3))
    for x, j in [(0.0, 0), (2.0, 0), (3.999999, 0), (4.0, 1), (5.5, 1), (6.999999, 1), (7.0, 2), (9.0, 2),
                 (10.0, 2)]:
        assert abs(density(m, th, x)[0] - child_p(j, x) / Z) < 1e-12 * child_p(j, x) / Z


def test_map_of_identical_children_is_the_child(oracle_mod):
    """Every range holding the same density gives Z = 1 and P = that density."""
    sp = copy.deepcopy(S.MAPPED)
    child = {"op": "gauss", "obs": "x", "par": ["m_mu", "m_sigma"]}
    sp["model"] = {"op": "map", "obs": "x", "bounds": [2.5, 7.5], "children": [child, child, child]}
    m = oracle_mod.Model(sp)
    one = copy.deepcopy(sp)
    one["model"] = child
    m1 = oracle_mod.Model(one)
    th = m.theta(S.MAPPED["truth"])
    x = np.linspace(0, 10, 41)
    assert np.allclose(m.logpdf(th, {"x": x}), m1.logpdf(th, {"x": x}), rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", ["mapped", "mapped_sum"])
def test_map_gradient_matches_finite_differences(oracle_mod, name):
    sp = S.workload(name)
    m = oracle_mod.Model(sp)
    rng = np.random.default_rng(4)
    th = m.theta(sp["truth"]) * (1 + 0.05 * rng.standard_normal(len(sp["params"])))
    d = {"x": rng.uniform(0.0, 10.0, 500)}
    v, g = m.nll(th, d, grad=True)
    gf = fd_grad(m, th, d, rel=1e-6)
    scale = np.abs(m.logpdf(th, d, grad_rows=True)[1]).sum(axis=0)
    assert np.all(np.abs(g - gf) <= 1e-7 * scale + 1e-7)


def test_map_sum_normalised(oracle_mod):
    m = oracle_mod.Model(S.MAPPED_SUM)
    th = m.theta(S.MAPPED_SUM["truth"])
    tot = integrate.quad(lambda x: density(m, th, x)[0], 0.0, 10.0, points=BOUNDS, epsabs=0, epsrel=1e-12,
                         limit=400)[0]
    assert abs(tot - 1.0) < 1e-11
