"""Pins of the oracle's binned metrics (the fit-manager metric switch of the
paper's "GooFit code" section, and binned fits such as its D*+ line-width
fit): binned NLL = -sum w ln P over bin centres, chi^2 = sum (w - K P)^2 /
max(w, 1) with K = (sum of weights) x bin volume.  The pins are independent
of the formulas: repeated events, an exactly integrable density, finite
differences and the statistics of fits to histograms."""
import numpy as np
import pytest

import synthgen as S
from helpers import get_spec

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

LINEAR = {
    "name": "linear",
    "obs": [("x", 0.0, 2.0)],
    "params": [("a1", 0.3, 0.05, 0.0, 0.0, False)],
    "truth": {"a1": 0.3},
    "model": {"op": "poly", "obs": "x", "par": ["a1"], "x0": 0.0},
}


def test_binned_nll_with_unit_weights_is_the_nll(oracle_mod):
    spec = S.C2
    m = oracle_mod.Model(spec)
    d = S.gen_c2(n=20_000, seed=61)
    th = m.theta(spec["truth"]) + np.array([0.01, 2e-4, 1e-4, 0.1])
    v, g = m.nll(th, d, grad=True)
    vb, gb = m.binned(th, d, np.ones(20_000), "bnll", 1.0, grad=True)
    assert abs(vb - v) <= 1e-12 * abs(v)
    assert np.allclose(gb, g, rtol=1e-11, atol=1e-9 * np.abs(g).max())


def test_binned_nll_with_integer_weights_is_the_nll_of_repeated_events(oracle_mod):
    spec = S.C2
    m = oracle_mod.Model(spec)
    d = S.gen_c2(n=3_000, seed=62)
    w = np.random.default_rng(63).integers(0, 5, 3_000).astype(np.float64)
    th = m.theta(spec["truth"])
    rep = {"x": np.repeat(d["x"], w.astype(np.int64))}
    v, g = m.nll(th, rep, grad=True)
    vb, gb = m.binned(th, d, w, "bnll", 1.0, grad=True)
    assert abs(vb - v) <= 1e-11 * abs(v)
    assert np.allclose(gb, g, rtol=1e-10, atol=1e-9 * np.abs(g).max())


def test_chi2_vanishes_at_exact_expected_counts(oracle_mod):
    """A linear density on [0, 2]: the midpoint rule integrates it exactly,
    so bin contents proportional to P at the centres are exactly the
    expected counts K P, and chi^2 and its gradient vanish at the truth."""
    m = oracle_mod.Model(LINEAR)
    nb = 40
    h = 2.0 / nb
    c = (np.arange(nb) + 0.5) * h
    th = m.theta(LINEAR["truth"])
    p = np.exp(m.logpdf(th, {"x": c}))
    assert abs(p.sum() * h - 1.0) < 1e-14
    w = 1000.0 * p
    v, g = m.binned(th, {"x": c}, w, "chi2", h, grad=True)
    assert v < 1e-20 and abs(g[0]) < 1e-9
    v2 = m.binned(th + 0.05, {"x": c}, w, "chi2", h)
    assert v2 > 1.0


@pytest.mark.parametrize("metric", ["bnll", "chi2"])
def test_binned_gradient_matches_finite_differences(oracle_mod, metric):
    spec = S.C2
    m = oracle_mod.Model(spec)
    x = S.gen_c2(n=200_000, seed=64)["x"]
    counts, edges = np.histogram(x, bins=500, range=(5.2, 5.3))
    c = 0.5 * (edges[1:] + edges[:-1])
    h = edges[1] - edges[0]
    th = m.theta(spec["truth"]) + np.array([0.01, 2e-4, 1e-4, 0.1])
    v, g = m.binned(th, {"x": c}, counts.astype(float), metric, h, grad=True)
    steps = np.array([1e-6, 1e-8, 1e-8, 1e-5])
    for j in range(4):
        tp, tm = th.copy(), th.copy()
        tp[j] += steps[j]
        tm[j] -= steps[j]
        fd = (m.binned(tp, {"x": c}, counts.astype(float), metric, h) -
              m.binned(tm, {"x": c}, counts.astype(float), metric, h)) / (2 * steps[j])
        assert abs(fd - g[j]) <= 1e-5 * max(abs(g[j]), 1.0) + 1e-6 * abs(v) / steps[j] * 1e-6


def test_binned_fits_recover_the_exponential_rate(oracle_mod):
    """10^6 exponential events in 100 bins: chi^2 and binned-likelihood fits
    find alpha within 3 sigma of the truth, chi^2_min / ndf is compatible
    with 1, and the two errors (up = 1 for chi^2, 0.5 for the likelihood)
    agree within 5 %."""
    spec = get_spec("c1")
    m = oracle_mod.Model(spec)
    x = S.gen_c1(n=1_000_000, seed=65)["x"]
    counts, edges = np.histogram(x, bins=100, range=(0.0, 10.0))
    c = {"x": 0.5 * (edges[1:] + edges[:-1])}
    h = edges[1] - edges[0]
    w = counts.astype(float)
    a0 = spec["truth"]["alpha"]
    rc = m.fit(c, binned={"weights": w, "metric": "chi2", "volume": h})
    rl = m.fit(c, binned={"weights": w, "metric": "bnll", "volume": h})
    for r in (rc, rl):
        assert abs(r["theta"][0] - a0) < 3 * r["errors"][0]
    ndf = 99
    assert abs(rc["nll"] / ndf - 1.0) < 5 * np.sqrt(2.0 / ndf)
    assert abs(rc["errors"][0] / rl["errors"][0] - 1.0) < 0.05
