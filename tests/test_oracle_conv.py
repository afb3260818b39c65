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
    f = lambda v: math.exp(m.logpdf(th, {"x": np.array([v])}, n_threads=1)[0])
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


# ------------------------------------------------------------------ nested: a resolution of several Gaussians
def _gmix_res(f="rf"):
    return {"op": "add", "par": [f], "children": [{"op": "gauss", "obs": "x", "par": ["r1", "s1"]},
                                                   {"op": "gauss", "obs": "x", "par": ["r2", "s2"]}]}


def test_gauss_smeared_by_a_gaussian_mixture_is_a_gaussian_mixture(oracle_mod):
    """G(m, s) convolved with f N(r1, s1) + (1 - f) N(r2, s2) (each normalised
    over the residual range, wide enough to hold them) is
    f N(m + r1, sqrt(s^2 + s1^2)) + (1 - f) N(m + r2, sqrt(s^2 + s2^2)),
    renormalised over the box: a fraction applied to the wrong component,
    a dropped component normalisation or variances added in the wrong
    place fail."""
    par = [("m", 5.0, 0.1, 0, 0, False), ("s", 0.6, 0.1, 0, 0, False), ("r1", 0.1, 0.1, 0, 0, False),
           ("s1", 0.3, 0.1, 0, 0, False), ("r2", -0.2, 0.1, 0, 0, False), ("s2", 0.8, 0.1, 0, 0, False),
           ("rf", 0.7, 0.1, 0, 1, False)]
    c = model(oracle_mod, par, conv(2000, -6.0, 6.0, {"op": "gauss", "obs": "x", "par": ["m", "s"]}, _gmix_res()))
    th = np.array([5.0, 0.6, 0.1, 0.3, -0.2, 0.8, 0.7])
    x = np.linspace(1.5, 8.5, 31)
    comps = [(0.7, 5.1, math.hypot(0.6, 0.3)), (0.3, 4.8, math.hypot(0.6, 0.8))]
    dens = sum(f * np.exp(-0.5 * ((x - mu) / sg) ** 2) / (sg * math.sqrt(2 * math.pi)) for f, mu, sg in comps)
    box = sum(f * 0.5 * (special.erf((10.0 - mu) / (math.sqrt(2) * sg)) - special.erf((0.0 - mu) / (math.sqrt(2) * sg)))
              for f, mu, sg in comps)
    ref = np.log(dens / box)
    assert np.max(np.abs(c.logpdf(th, {"x": x}) - ref)) < 1e-9


def test_a_mixture_with_one_component_is_that_component(oracle_mod):
    """f = 1: the mixture resolution is its first Gaussian, normalised over
    the residual range -- the same density as the plain Gaussian resolution
    (whose normalisation cancels in the convolution's Z)."""
    par = [("a", -0.4, 0.1, 0, 0, False), ("r1", 0.05, 0.1, 0, 0, False), ("s1", 0.3, 0.1, 0, 0, False),
           ("r2", -0.2, 0.1, 0, 0, False), ("s2", 0.8, 0.1, 0, 0, False), ("rf", 1.0, 0.1, 0, 1, False)]
    ex = {"op": "exp", "obs": "x", "par": ["a"]}
    mix = model(oracle_mod, par, conv(400, -2.0, 2.0, ex, _gmix_res()))
    one = model(oracle_mod, par, conv(400, -2.0, 2.0, ex, {"op": "gauss", "obs": "x", "par": ["r1", "s1"]}))
    th = np.array([-0.4, 0.05, 0.3, -0.2, 0.8, 1.0])
    x = np.linspace(0.05, 9.95, 37)
    assert np.max(np.abs(mix.logpdf(th, {"x": x}) - one.logpdf(th, {"x": x}))) < 1e-13


def test_mixture_resolution_workload_integrates_to_one_and_matches_fd(oracle_mod):
    sp = S.workload("conv_gmix")
    m = oracle_mod.Model(sp)
    th = m.theta(sp["truth"])
    f = lambda v: math.exp(m.logpdf(th, {"x": np.array([v])}, n_threads=1)[0])
    edges = np.linspace(0.0, 10.0, 81)
    tot = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11, limit=200)[0] for a, b in zip(edges[:-1], edges[1:]))
    assert abs(tot - 1.0) < 1e-8
    data = {"x": np.linspace(0.5, 9.5, 40)}
    v, g = m.nll(th, data, grad=True)
    fd = fd_grad(m, th, data)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-6 * np.abs(g).max())
