"""Pins of the oracle's trigonometric mixing terms (the time-dependent Dalitz
density with x free): the oscillating Gaussian-resolution convolution against
the Faddeeva-function closed form (a library routine), against its own x = 0
reduction to the closed-form E(t), its sigma -> 0 limit and its integrals
over t; the density's normalisation over t; and the gradient against finite
differences.  Each test names the mistake it would catch."""
import cmath
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import wofz

import synthgen as S

from test_oracle_pins import DZ, fd_grad, grid_cells


def closed_form(t, G, w, s):
    """int_0^inf e^{-(G - i w) u} N(t - u; 0, s) du via the Faddeeva function
    w(z) = e^{-z^2} erfc(-i z): 1/2 e^{-t^2/(2 s^2)} w(i xi) for Re xi > 0,
    else e^{z^2 s^2/2 - z t} - 1/2 e^{-t^2/(2 s^2)} w(-i xi), with z = G - i w
    and xi = (z s^2 - t)/(sqrt2 s)."""
    z = complex(G, -w)
    xi = (z * s * s - t) / (math.sqrt(2.0) * s)
    g = math.exp(-t * t / (2 * s * s))
    if xi.real > 0:
        return 0.5 * g * wofz(1j * xi)
    return cmath.exp(0.5 * z * z * s * s - z * t) - 0.5 * g * wofz(-1j * xi)


@pytest.mark.parametrize("t", [-0.5, -0.1, 0.0, 0.03, 0.41, 1.0, 2.5, 6.0])
@pytest.mark.parametrize("s", [0.02, 0.07, 0.2])
@pytest.mark.parametrize("w", [0.0, 0.012, 0.1, 0.6])
def test_oscillating_convolution_is_the_faddeeva_closed_form(oracle_mod, t, s, w):
    """A wrong sign of the sine part, a dropped e^{-G u} or a window that
    misses part of the Gaussian fails here."""
    G = 2.43
    o = oracle_mod.econv_osc(t, G, w, s)
    ref = closed_form(t, G, w, s)
    scale = oracle_mod.econv(t, G, s)
    assert abs(o[0] - ref.real) < 1e-12 * scale
    assert abs(o[1] - ref.imag) < 1e-12 * scale
    if w == 0.0:
        assert abs(o[0] - scale) < 1e-13 * scale and o[1] == 0.0


def test_oscillating_convolution_derivatives(oracle_mod):
    """d/dG and d/dw against central differences of the closed form (a
    swapped or sign-flipped derivative fails)."""
    for t, s, w in [(0.3, 0.05, 0.02), (-0.1, 0.1, 0.3), (2.0, 0.2, 0.05)]:
        G = 2.4
        o = oracle_mod.econv_osc(t, G, w, s)
        h = 1e-5
        dG = (closed_form(t, G + h, w, s) - closed_form(t, G - h, w, s)) / (2 * h)
        dw = (closed_form(t, G, w + h, s) - closed_form(t, G, w - h, s)) / (2 * h)
        sc = abs(oracle_mod.econv_dG(t, G, s)) + oracle_mod.econv(t, G, s)
        for got, ref in ((o[2], dG.real), (o[3], dG.imag), (o[4], dw.real), (o[5], dw.imag)):
            assert abs(got - ref) < 1e-8 * sc


def test_oscillating_convolution_limits_and_integrals(oracle_mod):
    """sigma -> 0 gives e^{-G t} (cos, sin)(w t); the integrals over t are
    G/(G^2 + w^2) and w/(G^2 + w^2) (a wrong frequency scale fails)."""
    G, w = 2.4, 0.35
    for t in (0.2, 1.1, 3.0):
        o = oracle_mod.econv_osc(t, G, w, 1e-5)
        assert abs(o[0] - math.exp(-G * t) * math.cos(w * t)) < 1e-9
        assert abs(o[1] - math.exp(-G * t) * math.sin(w * t)) < 1e-9
    s = 0.1
    ic = integrate.quad(lambda t: oracle_mod.econv_osc(t, G, w, s)[0], -2, 25, points=[0.0], epsrel=1e-12,
                        limit=400)[0]
    is_ = integrate.quad(lambda t: oracle_mod.econv_osc(t, G, w, s)[1], -2, 25, points=[0.0], epsrel=1e-12,
                         limit=400)[0]
    assert abs(ic - G / (G * G + w * w)) < 1e-10
    assert abs(is_ - w / (G * G + w * w)) < 1e-10


def _events(n, seed):
    rng = np.random.default_rng(seed)
    a, b, _ = grid_cells(dict(DZ, grid=80))
    m = oracle_mod_model("c4")
    keep = m.dalitz_amp2(m.theta(S.C4["truth"]), a, b) > 0
    idx = rng.choice(np.nonzero(keep)[0], n, replace=False)
    st = rng.uniform(0.02, 0.2, n)
    return {"s12": a[idx], "s13": b[idx], "sigma_t": st, "t": rng.exponential(0.41, n) + st * rng.standard_normal(n)}


_models = {}


def oracle_mod_model(name):
    from oracle import oracle as O
    if name not in _models:
        _models[name] = O.Model(S.workload(name))
    return _models[name]


def test_x_zero_reduces_to_the_hyperbolic_model(oracle_mod):
    """With x = 0 the model with the trigonometric terms (quadrature) is the
    x-free model (closed-form E): NLL and gradients agree."""
    m4, mx = oracle_mod_model("c4"), oracle_mod_model("c4x")
    d = _events(300, 7)
    th4 = m4.theta(S.C4["truth"])
    thx = np.append(th4, 0.0)
    v4, g4 = m4.nll(th4, d, grad=True)
    vx, gx = mx.nll(thx, d, grad=True)
    sc = np.abs(m4.logpdf(th4, d)).sum()
    assert abs(v4 - vx) < 1e-12 * sc
    gs = np.abs(m4.logpdf(th4, d, grad_rows=True)[1]).sum(axis=0)
    assert np.all(np.abs(g4 - gx[:-1]) <= 1e-11 * gs + 1e-12)


def test_mixing_density_time_integral(oracle_mod):
    """int dt of the density at fixed (s12, s13) equals the closed-form time
    integrals: a_c tau/(1-y^2) + a_0 tau/(1+x^2) + a_s y tau/(1-y^2)
    + b_s x tau/(1+x^2) (a wrong sign of the sin term, or of b_s, fails)."""
    m = oracle_mod_model("c4x")
    th = m.theta(S.C4X["truth"])
    th[-1] = 0.07  # a large x makes the trigonometric terms visible
    tau, y, x = th[-3], th[-2], th[-1]
    lnNT = m.node_lnnorm(m.root, th)[0]
    for s12, s13 in [(1.0, 1.2), (0.7, 2.0), (1.8, 0.9)]:
        a2 = m.dalitz_amp2(th, [s12], [s13])[0]
        b2 = m.dalitz_amp2(th, [s12], [s13], swapped=True)[0]
        X = m.dalitz_cross(th, [s12], [s13])[0]
        Y = m.dalitz_cross(th, [s12], [s13], imag=True)[0]
        st = 0.07
        f = lambda t: math.exp(m.logpdf(th, {"s12": np.array([s12]), "s13": np.array([s13]),
                                             "t": np.array([t]), "sigma_t": np.array([st])})[0] + lnNT)
        val = integrate.quad(f, -2.0, 15.0, points=[0.0], epsabs=0, epsrel=1e-11, limit=400)[0]
        ac, a0, as_, bs = 0.5 * (a2 + b2), 0.5 * (a2 - b2), -X, -Y
        ref = ac * tau / (1 - y * y) + a0 * tau / (1 + x * x) + as_ * y * tau / (1 - y * y) + bs * x * tau / (1 + x * x)
        assert abs(val - ref) < 1e-9 * (abs(ac) + abs(a0) + abs(as_) + abs(bs)) * tau


def test_mixing_unsmeared_rate_is_the_two_state_amplitude(oracle_mod):
    """The unsmeared rate equals |g+ A + g- Abar|^2 with g+- = (e^{-l1 t} +- e^{-l2 t})/2,
    l1 = Gamma (1 + y)/2 - i x Gamma/2, l2 = Gamma (1 - y)/2 + i x Gamma/2
    (fixes the sign conventions of the sinh and sin terms)."""
    m = oracle_mod_model("c4x")
    th = m.theta(S.C4X["truth"])
    th[-2], th[-1] = 0.04, 0.09
    tau, y, x = th[-3], th[-2], th[-1]
    G = 1 / tau
    pts = np.array([[1.0, 1.2], [0.7, 2.0], [1.8, 0.9]])
    ts = np.array([0.1, 0.8, 2.5])
    r = m.tddp_rate(th, pts[:, 0], pts[:, 1], ts)
    A = m.dalitz_amp(th, pts[:, 0], pts[:, 1])
    Ab = m.dalitz_amp(th, pts[:, 1], pts[:, 0])
    l1 = G * (1 + y) / 2 - 0.5j * x * G
    l2 = G * (1 - y) / 2 + 0.5j * x * G
    gp = 0.5 * (np.exp(-l1 * ts) + np.exp(-l2 * ts))
    gm = 0.5 * (np.exp(-l1 * ts) - np.exp(-l2 * ts))
    ref = np.abs(gp * A + gm * Ab) ** 2
    assert np.allclose(r, ref, rtol=1e-12, atol=0)


def test_mixing_gradient_matches_finite_differences(oracle_mod):
    m = oracle_mod_model("c4x")
    th = m.theta(S.C4X["truth"])
    th[-1] = 0.03
    rng = np.random.default_rng(9)
    th = th * (1 + 0.05 * rng.standard_normal(th.size))
    d = _events(300, 8)
    v, g = m.nll(th, d, grad=True)
    gf = fd_grad(m, th, d, rel=1e-6)
    scale = np.abs(m.logpdf(th, d, grad_rows=True)[1]).sum(axis=0)
    assert np.all(np.abs(g - gf) <= 1e-7 * scale + 1e-7)


def test_mixing_normalisation_is_the_grid_sum(oracle_mod):
    """N_T with x equals the midpoint sum over the Dalitz grid of the
    closed-form time integrals of the rate (a wrong sign or a missing Im J
    term in the normalisation fails)."""
    m = oracle_mod_model("c4x")
    th = m.theta(S.C4X["truth"])
    th[-2], th[-1] = 0.03, 0.08
    tau, y, x = th[-3], th[-2], th[-1]
    a, b, area = grid_cells(DZ)
    keep = m.dalitz_amp2(th, a, b) > 0
    a, b = a[keep], b[keep]
    a2 = m.dalitz_amp2(th, a, b)
    b2 = m.dalitz_amp2(th, a, b, swapped=True)
    X = m.dalitz_cross(th, a, b)
    Y = m.dalitz_cross(th, a, b, imag=True)
    per = (0.5 * (a2 + b2) * tau / (1 - y * y) + 0.5 * (a2 - b2) * tau / (1 + x * x)
           - X * y * tau / (1 - y * y) - Y * x * tau / (1 + x * x))
    ref = per.sum() * area
    lnNT = m.node_lnnorm(m.root, th)[0]
    assert abs(math.exp(lnNT) / ref - 1) < 1e-12
