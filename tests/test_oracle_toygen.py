"""Pins of the reference toy generator (oracle/toygen.py): the Philox4x32-10
stream against the generator's published known-answer vectors, the uniform
mapping, and the sampled distributions against their closed-form CDFs
(Kolmogorov-Smirnov), the mixture's CDF and the independence of a product's
factors.  A wrong round constant, a swapped word, an inverted CDF with a sign
or bound error, or a mixture choice against the wrong cumulative fraction
fails one of them."""
import json
import os

import numpy as np
import pytest
from scipy import special, stats

import synthgen as S
from oracle import toygen as T

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_philox_known_answer_vectors():
    kat = json.load(open(GOLD))
    for v in kat["vectors"]:
        out = T.philox4x32_10([[int(w, 16) for w in v["ctr"]]], [int(w, 16) for w in v["key"]])[0]
        assert [int(w) for w in out] == [int(w, 16) for w in v["out"]]


def test_uniform_mapping_and_stream_layout():
    idx = np.arange(200_000)
    u0 = T.uniforms(idx, 12345, 0)
    u1 = T.uniforms(idx, 12345, 1)
    u2 = T.uniforms(idx, 12345, 2)
    assert np.all((u0 > 0) & (u0 < 1))
    for u in (u0, u1, u2):
        assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(u0, u1)[0, 1]) < 0.01 and abs(np.corrcoef(u0, u2)[0, 1]) < 0.01
    # numbers 0 and 1 share a block (words 0-1 and 2-3); 2 is the next block
    w = T.philox4x32_10([[5, 0, 0, 0]], [12345, 0])[0]
    bits = ((int(w[2]) << 32) | int(w[3])) >> 11
    assert T.uniforms(np.array([5]), 12345, 1)[0] == (bits + 0.5) * 2.0 ** -53
    # an event's numbers do not depend on the others, and the seed's high word matters
    assert np.array_equal(T.uniforms(idx[1000:1010], 12345, 0), u0[1000:1010])
    assert not np.array_equal(T.uniforms(idx[:10], 12345 + (1 << 32), 0), u0[:10])


def _cdf_exp(x, a, b, al):
    return np.expm1(al * (x - a)) / np.expm1(al * (b - a))


def test_exponential_matches_closed_form_cdf():
    sp = S.workload("c1")
    x = T.generate(sp, [-0.5], 100_000, 7)["x"]
    assert x.min() >= 0.0 and x.max() <= 10.0
    assert stats.kstest(x, lambda v: _cdf_exp(v, 0.0, 10.0, -0.5)).pvalue > 1e-3
    # positive rate and the flat limit
    x = T.generate(sp, [0.3], 50_000, 8)["x"]
    assert stats.kstest(x, lambda v: _cdf_exp(v, 0.0, 10.0, 0.3)).pvalue > 1e-3
    x = T.generate(sp, [0.0], 50_000, 9)["x"]
    assert stats.kstest(x, stats.uniform(0.0, 10.0).cdf).pvalue > 1e-3


def test_truncated_gaussian_matches_closed_form_cdf():
    sp = {"obs": [("x", 0.0, 10.0)], "params": [("m", 0, 1, 0, 0, False), ("s", 1, 1, 0, 0, False)],
          "model": {"op": "gauss", "obs": "x", "par": ["m", "s"]}}
    for mu, sg in [(6.0, 1.2), (9.5, 2.0), (0.0, 0.3)]:
        x = T.generate(sp, [mu, sg], 60_000, 10)["x"]
        d = stats.truncnorm((0.0 - mu) / sg, (10.0 - mu) / sg, loc=mu, scale=sg)
        assert stats.kstest(x, d.cdf).pvalue > 1e-3, (mu, sg)


def test_mixture_matches_its_cdf():
    sp = S.workload("c2")
    th = np.array([0.3, 5.28, 0.003, -2.0])
    x = T.generate(sp, th, 200_000, 11)["x"]
    g = stats.truncnorm((5.2 - 5.28) / 0.003, (5.3 - 5.28) / 0.003, loc=5.28, scale=0.003)
    cdf = lambda v: 0.3 * g.cdf(v) + 0.7 * _cdf_exp(v, 5.2, 5.3, -2.0)
    assert stats.kstest(x, cdf).pvalue > 1e-3
    # fraction of events within 5 sigma of the peak: f plus the exponential's share there
    near = np.abs(x - 5.28) < 0.015
    p = 0.3 * (g.cdf(5.295) - g.cdf(5.265)) + 0.7 * (_cdf_exp(5.295, 5.2, 5.3, -2) - _cdf_exp(5.265, 5.2, 5.3, -2))
    assert abs(near.mean() - p) < 4 * np.sqrt(p * (1 - p) / x.size)


def test_product_factors_are_independent_with_their_marginals():
    sp = S.workload("listing2")
    d = T.generate(sp, [-0.5, -1.0], 100_000, 12)
    assert stats.kstest(d["x"], lambda v: _cdf_exp(v, 0.0, 10.0, -0.5)).pvalue > 1e-3
    assert stats.kstest(d["y"], lambda v: _cdf_exp(v, 0.0, 10.0, -1.0)).pvalue > 1e-3
    assert abs(stats.spearmanr(d["x"], d["y"])[0]) < 0.02


def test_unsupported_leaf_is_refused():
    with pytest.raises(ValueError):
        T.generate(S.workload("mapped"), np.zeros(len(S.workload("mapped")["params"])), 10, 1)


def test_accept_reject_layout_and_distribution():
    """A flat density under an envelope equal to it accepts every first
    candidate (pins the candidate's uniform numbers); an exponential follows
    its closed-form CDF; an envelope below the density is refused."""
    sp = S.workload("c1")
    x = T.generate_ar(sp, [0.0], 1000, 3, 0.1)["x"]
    assert np.array_equal(x, 0.0 + T.uniforms(np.arange(1000), 3, 0) * 10.0)
    x = T.generate_ar(sp, [-0.5], 40_000, 4, 0.6)["x"]
    assert stats.kstest(x, lambda v: _cdf_exp(v, 0.0, 10.0, -0.5)).pvalue > 1e-3
    with pytest.raises(ValueError):
        T.generate_ar(sp, [-0.5], 1000, 4, 0.3)


def test_accept_reject_dalitz_moments():
    """Dalitz events: inside the plot, and the s12 and s13 means agree with
    the density-weighted means over a fine grid within 4 standard errors."""
    from oracle import oracle as O
    sp = S.workload("c3")
    m = O.Model(sp)
    th = m.theta(sp["truth"])
    lo, hi = S.dalitz_box()
    G = 400
    c = lo + (np.arange(G) + 0.5) * (hi - lo) / G
    a, b = np.meshgrid(c, c, indexing="ij")
    p = np.exp(m.logpdf(th, {"s12": a.ravel(), "s13": b.ravel()}))
    d = T.generate_ar(sp, th, 20_000, 6, 1.5 * p.max())
    assert all(O.inside(sp["model"]["dalitz"], u, v) for u, v in zip(d["s12"][:500], d["s13"][:500]))
    for k, grid in (("s12", a.ravel()), ("s13", b.ravel())):
        mean = np.sum(p * grid) / np.sum(p)
        sd = np.sqrt(np.sum(p * (grid - mean) ** 2) / np.sum(p))
        assert abs(d[k].mean() - mean) < 4 * sd / np.sqrt(d[k].size), k
