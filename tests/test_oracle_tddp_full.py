"""Pins of the oracle's full time-dependent model (section "Results": the
mixing fit with 16 complex amplitudes, complex q/p and floating resonance
masses and widths) against what does not depend on its own formulas:
finite differences, the fixed-shape model it must reduce to, two separate
routes to the normalisation, the no-mixing limit where q/p drops out, and
the time integral of the density by quadrature.

Each test names the plausible oracle mistake it would catch."""
import copy
import math

import numpy as np
import pytest

import synthgen as S


def full_spec(grid=60):
    return S.configs._full_model(grid=grid)


def points(spec, n, seed):
    """n points uniform over the Dalitz plot with exponential decay times
    and sigma_t ~ U[0.02, 0.2] (pins need no particular distribution)."""
    from oracle import oracle as O
    dz = spec["model"]["dalitz"]
    lo, hi = S.dalitz_box()
    rng = np.random.default_rng(seed)
    a, b = [], []
    while len(a) < n:
        u, v = rng.uniform(lo, hi, 2)
        if O.inside(dz, u, v):
            a.append(u)
            b.append(v)
    t = rng.exponential(0.41, n) + rng.normal(0.0, 0.05, n)
    return {"s12": np.array(a), "s13": np.array(b), "t": t, "sigma_t": rng.uniform(0.02, 0.2, n)}


def theta_off(m, spec, seed=3):
    """A parameter point away from the truth in every direction (q/p not 1,
    x and y larger than physical so that their terms weigh in)."""
    rng = np.random.default_rng(seed)
    th = m.theta(spec["truth"])
    th[:30] *= 1.0 + 0.2 * rng.standard_normal(30)
    i = m.par_names.index
    th[i("tau")], th[i("y")], th[i("x")] = 0.43, 0.06, 0.05
    th[i("qp_mag")], th[i("qp_phase")] = 0.85, 0.4
    th[i("rho_m0")], th[i("rho_g0")] = 0.781, 0.143
    th[i("kst_m0")], th[i("kst_g0")] = 0.889, 0.054
    return th


def test_resonance_shape_derivatives_fd(oracle_mod):
    """dA/dm0 and dA/dGamma0 against central differences of the amplitude
    for every spin and pair; catches a dropped dependence of q0 or of the
    barrier factor on m0, or a wrong power of q/q0."""
    dz = S.DALITZ_KINEMATICS
    pts = [(1.0, 1.4), (0.7, 2.2), (1.8, 0.9), (2.3, 0.8)]
    for ch, m0, g0, J in [("23", 0.775, 0.149, 1), ("23", 0.5, 0.4, 0), ("23", 1.275, 0.185, 2),
                          ("12", 0.892, 0.05, 1), ("13", 1.43, 0.1, 2), ("12", 1.425, 0.27, 0)]:
        for s12, s13 in pts:
            if not oracle_mod.inside(dz, s12, s13):
                continue
            a, dm, dg = oracle_mod.res_amp_d(dz, ch, m0, g0, J, s12, s13)
            h = 1e-6
            fm = (oracle_mod.res_amp_d(dz, ch, m0 + h, g0, J, s12, s13)[0] -
                  oracle_mod.res_amp_d(dz, ch, m0 - h, g0, J, s12, s13)[0]) / (2 * h)
            fg = (oracle_mod.res_amp_d(dz, ch, m0, g0 + h, J, s12, s13)[0] -
                  oracle_mod.res_amp_d(dz, ch, m0, g0 - h, J, s12, s13)[0]) / (2 * h)
            assert abs(dm - fm) <= 1e-6 * max(abs(fm), abs(a)), (ch, J, s12, s13, dm, fm)
            assert abs(dg - fg) <= 1e-6 * max(abs(fg), abs(a)), (ch, J, s12, s13, dg, fg)


def test_reduces_to_fixed_shape_model(oracle_mod):
    """With q/p = 1 and the floating masses and widths at their fixed values
    the full model equals the plain time-dependent model with x: same NLL
    and the same derivatives in every shared parameter; catches q/p or the
    shape parameters entering where they should be neutral."""
    spec = full_spec()
    m = oracle_mod.Model(spec)
    th = m.theta(spec["truth"])
    i = m.par_names.index
    th[i("qp_mag")], th[i("qp_phase")] = 1.0, 0.0
    th[i("y")], th[i("x")] = 0.03, 0.02
    plain = copy.deepcopy(spec)
    node = plain["model"]
    for r in node["dalitz"]["resonances"]:
        r.pop("float", None)
    node.pop("qp")
    node["par"] = node["par"][:30] + ["tau", "y", "x"]
    plain["params"] = [p for p in spec["params"] if p[0] in node["par"]]
    mp_ = oracle_mod.Model(plain)
    d = points(spec, 400, 1)
    v, g = m.nll(th, d, grad=True)
    thp = np.array([th[i(n)] for n in mp_.par_names])
    vp, gp = mp_.nll(thp, d, grad=True)
    assert abs(v - vp) <= 1e-12 * abs(vp)
    for j, n in enumerate(mp_.par_names):
        assert abs(g[i(n)] - gp[j]) <= 1e-9 * max(1.0, np.abs(gp).max()), n


def test_direct_grid_sum_equals_matrix_normalisation(oracle_mod):
    """With fixed shapes the normalisation comes from grid matrices (c^H I c
    forms scaled by |q/p|^2 and q/p); the cell-by-cell grid sum of the
    time-integrated rate at theta must give the same ln N and gradient;
    catches a wrong q/p scaling of the conjugate or cross matrices, or a
    sign in a time integral."""
    spec = full_spec(grid=80)
    node = spec["model"]
    for r in node["dalitz"]["resonances"]:
        r.pop("float", None)
    keep = node["par"][:35]
    node["par"] = keep
    spec["params"] = [p for p in spec["params"] if p[0] in keep]
    spec["truth"] = {k: v for k, v in spec["truth"].items() if k in keep}
    m = oracle_mod.Model(spec)
    th = m.theta(spec["truth"])
    rng = np.random.default_rng(5)
    th[:30] *= 1.0 + 0.2 * rng.standard_normal(30)
    i = m.par_names.index
    th[i("y")], th[i("x")], th[i("qp_mag")], th[i("qp_phase")] = 0.05, -0.04, 0.8, -0.6
    nid = m.root
    l1, g1 = m.node_lnnorm(nid, th)
    m.set_direct_norm(True)
    l2, g2 = m.node_lnnorm(nid, th)
    m.set_direct_norm(False)
    assert abs(l1 - l2) <= 1e-13 * abs(l1)
    assert np.abs(g1 - g2).max() <= 1e-12 * np.abs(g1).max()


def test_gradient_fd(oracle_mod):
    """The analytic gradient (coefficients, tau, y, x, |q/p|, arg q/p and the
    floating masses and widths, each through the events and the
    normalisation) against central differences of the oracle's NLL."""
    spec = full_spec()
    m = oracle_mod.Model(spec)
    th = theta_off(m, spec)
    d = points(spec, 300, 2)
    v, g = m.nll(th, d, grad=True)
    for j in range(th.size):
        h = 1e-6 * max(abs(th[j]), 0.01)
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (m.nll(tp, d) - m.nll(tm, d)) / (2 * h)
        assert abs(g[j] - fd) <= 2e-6 * max(1.0, abs(fd)), (m.par_names[j], g[j], fd)


def test_no_mixing_q_over_p_drops_out(oracle_mod):
    """At x = y = 0 the rate is |A|^2 e^{-t/tau} (convolved): q/p must not
    change the NLL, and its derivatives vanish; catches q/p multiplying A
    instead of Abar or entering the normalisation outside the mixing
    terms."""
    spec = full_spec()
    m = oracle_mod.Model(spec)
    th = theta_off(m, spec)
    i = m.par_names.index
    th[i("x")], th[i("y")] = 0.0, 0.0
    d = points(spec, 300, 4)
    v1, g1 = m.nll(th, d, grad=True)
    th2 = th.copy()
    th2[i("qp_mag")], th2[i("qp_phase")] = 1.3, -0.9
    v2 = m.nll(th2, d)
    assert abs(v1 - v2) <= 1e-12 * abs(v1)
    assert abs(g1[i("qp_mag")]) <= 1e-9 and abs(g1[i("qp_phase")]) <= 1e-9


def test_density_integrates_to_one(oracle_mod):
    """Sum over the grid cells (inside the plot, times the cell area) of the
    time integral of the density by Gauss-Legendre quadrature equals 1 at a
    point with q/p, x, y and the floating shapes all away from their
    defaults; catches per-event and normalisation terms that disagree (the
    two are separate code)."""
    spec = full_spec(grid=40)
    m = oracle_mod.Model(spec)
    th = theta_off(m, spec)
    dz = spec["model"]["dalitz"]
    lo12 = (dz["m1"] + dz["m2"]) ** 2
    hi12 = (dz["M"] - dz["m3"]) ** 2
    lo13 = (dz["m1"] + dz["m3"]) ** 2
    hi13 = (dz["M"] - dz["m2"]) ** 2
    G = dz["grid"]
    h12, h13 = (hi12 - lo12) / G, (hi13 - lo13) / G
    c12 = lo12 + (np.arange(G) + 0.5) * h12
    c13 = lo13 + (np.arange(G) + 0.5) * h13
    a, b = np.meshgrid(c12, c13, indexing="ij")
    a, b = a.ravel(), b.ravel()
    from oracle import oracle as O
    ins = np.array([O.inside(dz, u, v) for u, v in zip(a, b)])
    a, b = a[ins], b[ins]
    # t over [-1.5, 40]: composite 16-point Gauss-Legendre, 200 panels
    xg, wg = np.polynomial.legendre.leggauss(16)
    edges = np.linspace(-1.5, 40.0, 201)
    tt = np.concatenate([0.5 * (e1 - e0) * xg + 0.5 * (e1 + e0) for e0, e1 in zip(edges[:-1], edges[1:])])
    wt = np.concatenate([0.5 * (e1 - e0) * wg for e0, e1 in zip(edges[:-1], edges[1:])])
    for sig in (0.03, 0.15):
        d = {"s12": np.repeat(a, tt.size), "s13": np.repeat(b, tt.size), "t": np.tile(tt, a.size),
             "sigma_t": np.full(a.size * tt.size, sig)}
        p = np.exp(m.logpdf(th, d)).reshape(a.size, tt.size)
        tot = float((p @ wt).sum()) * h12 * h13
        assert abs(tot - 1.0) <= 1e-12, (sig, tot)
