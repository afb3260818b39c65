"""Pins of the reference oracle against what mathematics fixes independently
of it: closed forms evaluated in high precision from the textbook integrals,
numerical quadrature, textbook maximum-likelihood special cases, finite
differences, and reductions of composite nodes to simpler ones.

Each test names the plausible oracle mistake it would catch."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import synthgen as S


def spec1(model, obs, params):
    return {"obs": obs, "params": params, "model": model}


def fd_grad(m, th, data, rel=1e-6):
    g = np.zeros_like(th)
    for j in range(th.size):
        h = rel * max(abs(th[j]), 1e-3)
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        g[j] = (m.nll(tp, data) - m.nll(tm, data)) / (2 * h)
    return g


# ------------------------------------------------------------------ EXP
def test_exp_closed_form_mpmath(oracle_mod):
    """NLL of e^{alpha x}/int_a^b e^{alpha x} written from the raw integral in
    30-digit arithmetic; catches a wrong normalisation, sign or offset."""
    m = oracle_mod.Model(S.C1)
    x = S.gen_c1(n=2000, seed=123)["x"]
    mp.mp.dps = 30
    sx = mp.fsum([mp.mpf(float(v)) for v in x])
    for alpha in (-2.0, -0.5, -1e-7, 0.0, 1e-9, 0.3, 1.0):
        a = mp.mpf(alpha)
        if alpha == 0.0:
            lnN = mp.log(10)
            dlnN = mp.mpf(5)
        else:
            N = (mp.exp(a * 10) - 1) / a
            lnN = mp.log(N)
            dlnN = mp.diff(lambda z: mp.log((mp.exp(z * 10) - 1) / z), a)
        ref = -a * sx + len(x) * lnN
        gref = -sx + len(x) * dlnN
        v, g = m.nll([alpha], {"x": x}, grad=True)
        assert abs(v - float(ref)) <= 1e-13 * abs(float(ref)), alpha
        assert abs(g[0] - float(gref)) <= 1e-10 * float(sx), alpha


def test_exp_normalised_by_quadrature(oracle_mod):
    """int P dx = 1 by adaptive quadrature of the oracle's own log-density."""
    m = oracle_mod.Model(S.C1)
    for alpha in (-3.0, -0.5, 0.2):
        f = lambda x: math.exp(m.logpdf([alpha], {"x": np.array([x])})[0])
        val, err = integrate.quad(f, 0.0, 10.0, epsabs=0, epsrel=1e-13, limit=200)
        assert abs(val - 1.0) < 1e-12


def test_exp_psi_series_vs_mpmath(oracle_mod):
    """psi(z) = 1/(1-e^{-z}) - 1/z near 0 (series branch) and above it."""
    mp.mp.dps = 40
    for z in (-5e-3, -1e-6, 1e-9, 3e-3, 9.99e-3, 1.01e-2, 0.5, -20.0, 40.0):
        zz = mp.mpf(z)
        ref = 1 / (1 - mp.exp(-zz)) - 1 / zz
        assert abs(oracle_mod.psi(z) - float(ref)) < 3e-14 * max(1.0, abs(float(ref)))


def test_exp_fit_errors_match_fisher_information(oracle_mod):
    """The fitted error equals the closed-form Fisher information of the
    truncated exponential, 1/sqrt(n Var(x)), at the fitted alpha."""
    m = oracle_mod.Model(S.C1)
    d = S.gen_c1(n=20000, seed=9)
    r = m.fit(d)
    a, L, n = r["theta"][0], 10.0, 20000
    var = 1 / a**2 - L**2 * math.exp(a * L) / (math.expm1(a * L)) ** 2
    assert abs(r["errors"][0] - 1 / math.sqrt(n * var)) < 1e-5 * r["errors"][0]
    # MLE condition for an exponential family: model mean equals sample mean
    mean = integrate.quad(lambda x: x * math.exp(m.logpdf([a], {"x": np.array([x])})[0]), 0, 10,
                          epsrel=1e-13)[0]
    assert abs(mean - d["x"].mean()) < 1e-9


# ------------------------------------------------------------------ GAUSS
GSPEC = spec1({"op": "gauss", "obs": "x", "par": ["mu", "sigma"]}, [("x", 5.2, 5.3)],
              [("mu", 5.28, 0.001, 5.2, 5.3, False), ("sigma", 0.003, 0.0005, 1e-4, 0.05, False)])


@pytest.mark.parametrize("mu,sigma", [(5.28, 0.003), (5.2005, 0.004), (5.25, 0.06), (5.31, 0.01)])
def test_gauss_normalised_by_quadrature(oracle_mod, mu, sigma):
    m = oracle_mod.Model(GSPEC)
    f = lambda x: math.exp(m.logpdf([mu, sigma], {"x": np.array([x])})[0])
    pts = [p for p in (mu - 5 * sigma, mu, mu + 5 * sigma) if 5.2 < p < 5.3]
    val = integrate.quad(f, 5.2, 5.3, points=pts or None, epsabs=0, epsrel=1e-13, limit=400)[0]
    assert abs(val - 1.0) < 1e-11


def test_gauss_wide_range_is_textbook_normal(oracle_mod):
    """On a range of +-40 sigma the normalisation is sigma sqrt(2 pi)."""
    spec = spec1({"op": "gauss", "obs": "x", "par": ["mu", "sigma"]}, [("x", -40.0, 40.0)],
                 [("mu", 0.3, 0.1, -5, 5, False), ("sigma", 1.0, 0.1, 0.1, 5, False)])
    m = oracle_mod.Model(spec)
    lnN, d = m.node_lnnorm(m.root, np.array([0.3, 1.3]))
    assert abs(lnN - math.log(1.3 * math.sqrt(2 * math.pi))) < 1e-15
    assert abs(d[0]) < 1e-15 and abs(d[1] - 1 / 1.3) < 1e-14


def test_gauss_mle_is_sample_mean_and_rms(oracle_mod):
    """Textbook MLE of a normal sample (negligible truncation): mu = mean,
    sigma = rms about the mean."""
    spec = spec1({"op": "gauss", "obs": "x", "par": ["mu", "sigma"]}, [("x", -60.0, 60.0)],
                 [("mu", 0.5, 0.1, -5, 5, False), ("sigma", 1.5, 0.1, 0.1, 5, False)])
    m = oracle_mod.Model(spec)
    x = np.random.default_rng(4).normal(0.2, 1.1, 5000)
    r = m.fit({"x": x})
    assert abs(r["theta"][0] - x.mean()) < 1e-9
    assert abs(r["theta"][1] - x.std()) < 1e-9
    assert abs(r["errors"][0] - x.std() / math.sqrt(x.size)) < 1e-6 * r["errors"][0]


# ------------------------------------------------------------------ POLY
def test_poly_normalisation_gauss_legendre_and_uniform(oracle_mod):
    spec = spec1({"op": "poly", "obs": "x", "par": ["a1", "a2", "a3"], "x0": 1.0}, [("x", -1.0, 3.0)],
                 [("a1", 0.2, 0.1, 0, 0, False), ("a2", 0.3, 0.1, 0, 0, False),
                  ("a3", -0.05, 0.01, 0, 0, False)])
    m = oracle_mod.Model(spec)
    th = np.array([0.2, 0.3, -0.05])
    xg, wg = np.polynomial.legendre.leggauss(4)  # exact for degree <= 7
    x = 1.0 + 2.0 * xg
    p = np.exp(m.logpdf(th, {"x": x}))
    assert abs(2.0 * (wg * p).sum() - 1.0) < 1e-14
    # degree 0 (all coefficients zero) is the uniform density 1/L
    lp = m.logpdf(np.zeros(3), {"x": np.array([-0.5, 2.9])})
    assert np.allclose(lp, -math.log(4.0), rtol=0, atol=1e-15)
    # a non-positive polynomial at an event gives NLL = +inf
    assert m.nll(np.array([-2.0, 0.0, 0.0]), {"x": np.array([2.5])}) == math.inf


# ------------------------------------------------------------------ ADD / PROD
def test_add_normalised_and_reduces_to_child(oracle_mod):
    m = oracle_mod.Model(S.C2)
    for th in ([0.3, 5.28, 0.003, -2.0], [0.7, 5.21, 0.02, 3.0]):
        f = lambda x: math.exp(m.logpdf(th, {"x": np.array([x])})[0])
        val = integrate.quad(f, 5.2, 5.3, points=[th[1]], epsabs=0, epsrel=1e-13, limit=400)[0]
        assert abs(val - 1.0) < 1e-11
    # f = 1: the sum is its first child
    g = oracle_mod.Model(GSPEC)
    x = S.gen_c2(n=3000, seed=5)["x"]
    assert abs(m.nll([1.0, 5.281, 0.0031, -2.0], {"x": x}) - g.nll([5.281, 0.0031], {"x": x})) < 1e-9
    # f = 0: the sum is its last child
    e = oracle_mod.Model(spec1({"op": "exp", "obs": "x", "par": ["beta"]}, [("x", 5.2, 5.3)],
                               [("beta", -1.0, 0.1, -10, 10, False)]))
    assert abs(m.nll([0.0, 5.281, 0.0031, -2.0], {"x": x}) - e.nll([-2.0], {"x": x})) < 1e-9


def test_prod_listing2_separates(oracle_mod):
    """Listing 2: the 2-D product NLL is the sum of the two 1-D NLLs and the
    product density integrates to one."""
    m = oracle_mod.Model(S.LISTING2)
    d = S.gen_listing2(n=4000, seed=3)
    ex = oracle_mod.Model(spec1({"op": "exp", "obs": "x", "par": ["a"]}, [("x", 0.0, 10.0)],
                                [("a", -1, 0.1, -10, 10, False)]))
    th = np.array([-0.45, -1.1])
    v, g = m.nll(th, d, grad=True)
    vx, gx = ex.nll([th[0]], {"x": d["x"]}, grad=True)
    vy, gy = ex.nll([th[1]], {"x": d["y"]}, grad=True)
    assert abs(v - (vx + vy)) < 1e-10 * abs(v)
    assert abs(g[0] - gx[0]) < 1e-9 and abs(g[1] - gy[0]) < 1e-9
    f = lambda y, x: math.exp(m.logpdf(th, {"x": np.array([x]), "y": np.array([y])})[0])
    val = integrate.dblquad(f, 0, 10, 0, 10, epsabs=1e-12, epsrel=1e-11)[0]
    assert abs(val - 1.0) < 1e-10


@pytest.mark.parametrize("cfg", ["c1", "c2", "listing2"])
def test_gradient_matches_finite_differences(oracle_mod, cfg):
    spec = S.workload(cfg)
    m = oracle_mod.Model(spec)
    gen = {"c1": S.gen_c1, "c2": S.gen_c2, "listing2": S.gen_listing2}[cfg]
    d = gen(n=3000, seed=21)
    th = m.theta() * 1.01
    v, g = m.nll(th, d, grad=True)
    gf = fd_grad(m, th, d)
    scale = np.abs(m.logpdf(th, d, grad_rows=True)[1]).sum(axis=0)
    assert np.all(np.abs(g - gf) <= 1e-7 * scale + 1e-6)


# ------------------------------------------------------------------ time convolution
def test_erfcx_vs_mpmath(oracle_mod):
    mp.mp.dps = 40
    for x in (0.0, 0.1, 1.0, 3.0, 4.99, 5.0, 5.01, 7.5, 12.0, 30.0, 1e3, 1e6):
        ref = mp.exp(mp.mpf(x) ** 2) * mp.erfc(mp.mpf(x))
        assert abs(oracle_mod.erfcx(x) - float(ref)) < 4e-15 * float(ref), x


@pytest.mark.parametrize("t,G,s", [(0.3, 2.44, 0.05), (-0.15, 2.44, 0.05), (-0.4, 2.0, 0.05),
                                   (1.5, 2.5, 0.2), (0.0, 2.4, 0.02), (-0.2, 2.4, 0.02),
                                   (0.05, 10.0, 0.2)])
def test_econv_is_the_convolution(oracle_mod, t, G, s):
    """E(t) = int_0^inf e^{-G u} N(t-u; 0, s) du by quadrature."""
    f = lambda u: math.exp(-G * u) * math.exp(-0.5 * ((t - u) / s) ** 2) / (s * math.sqrt(2 * math.pi))
    ref = integrate.quad(f, 0.0, max(t, 0.0) + 40 * s + 40 / G, points=[max(t, 0.0)], epsabs=0,
                         epsrel=1e-13, limit=400)[0]
    assert abs(oracle_mod.econv(t, G, s) - ref) < 1e-11 * ref
    h = 1e-6 * G
    fd = (oracle_mod.econv(t, G + h, s) - oracle_mod.econv(t, G - h, s)) / (2 * h)
    assert abs(oracle_mod.econv_dG(t, G, s) - fd) < 1e-7 * max(abs(fd), ref)


def test_econv_moments(oracle_mod):
    """int E = 1/G, mean 1/G, variance 1/G^2 + s^2; s -> 0 gives e^{-G t}."""
    G, s = 2.4, 0.1
    f = lambda t: oracle_mod.econv(t, G, s)
    m0 = integrate.quad(f, -3, 20, points=[0.0], epsrel=1e-13, limit=400)[0]
    m1 = integrate.quad(lambda t: t * f(t), -3, 20, points=[0.0], epsrel=1e-13, limit=400)[0]
    m2 = integrate.quad(lambda t: t * t * f(t), -3, 20, points=[0.0], epsrel=1e-13, limit=400)[0]
    assert abs(m0 * G - 1) < 1e-11
    mean = m1 / m0
    assert abs(mean - 1 / G) < 1e-10
    assert abs(m2 / m0 - mean**2 - (1 / G**2 + s**2)) < 1e-10
    assert abs(oracle_mod.econv(0.7, G, 1e-6) - math.exp(-G * 0.7)) < 1e-12


# ------------------------------------------------------------------ Dalitz kinematics
DZ = S.C3["model"]["dalitz"]


def pdg_s13_limits(s12, kin):
    """s13 range at fixed s12 from the standard three-body formulae."""
    M, m1, m2, m3 = kin["M"], kin["m1"], kin["m2"], kin["m3"]
    m12 = math.sqrt(s12)
    E1 = (s12 - m2**2 + m1**2) / (2 * m12)
    E3 = (M**2 - s12 - m3**2) / (2 * m12)
    p1 = math.sqrt(max(E1**2 - m1**2, 0))
    p3 = math.sqrt(max(E3**2 - m3**2, 0))
    return (E1 + E3) ** 2 - (p1 + p3) ** 2, (E1 + E3) ** 2 - (p1 - p3) ** 2


def test_dalitz_area_and_membership(oracle_mod):
    lo, hi = S.dalitz_box()
    area = integrate.quad(lambda s: np.subtract(*pdg_s13_limits(s, DZ)[::-1]), lo, hi,
                          epsabs=0, epsrel=1e-13, limit=400)[0]
    assert abs(area - 3.1389159334507) < 1e-10
    m = oracle_mod.Model(S.C3)
    I = m.dalitz_matrix(0)
    assert abs(I[0, 0].real - area) < 2e-5 * area  # grid area converges to the true area
    rng = np.random.default_rng(0)
    for a, b in zip(lo + (hi - lo) * rng.random(4000), lo + (hi - lo) * rng.random(4000)):
        smin, smax = pdg_s13_limits(a, DZ)
        if min(abs(b - smin), abs(b - smax)) < 1e-9:
            continue
        assert oracle_mod.inside(DZ, a, b) == (smin <= b <= smax)


def pdg_line(sAB, ch, kin):
    """Endpoints in s_AC at fixed s_AB and the momenta p (bachelor) and q
    (daughter) in the AB rest frame."""
    M = kin["M"]
    mA, mB, mC = {"23": (kin["m2"], kin["m3"], kin["m1"]), "12": (kin["m1"], kin["m2"], kin["m3"]),
                  "13": (kin["m1"], kin["m3"], kin["m2"])}[ch]
    r = math.sqrt(sAB)
    EA = (sAB - mB**2 + mA**2) / (2 * r)
    EC = (M**2 - sAB - mC**2) / (2 * r)
    q = math.sqrt(EA**2 - mA**2)
    p = math.sqrt(EC**2 - mC**2)
    return (EA + EC) ** 2 - (q + p) ** 2, (EA + EC) ** 2 - (q - p) ** 2, p, q


def to_s12_s13(ch, sAB, sAC, kin):
    tot = kin["M"] ** 2 + kin["m1"] ** 2 + kin["m2"] ** 2 + kin["m3"] ** 2
    if ch == "23":      # AC = (2,1) -> s12
        s12 = sAC
        return s12, tot - sAB - s12
    if ch == "12":      # AC = (1,3) -> s13
        return sAB, sAC
    return sAC, sAB     # ch 13: AC = (1,2) -> s12


@pytest.mark.parametrize("ch,m0,g0", [("23", 0.775, 0.149), ("12", 0.892, 0.05), ("13", 1.1, 0.2)])
def test_breit_wigner_and_barrier_at_pole(oracle_mod, ch, m0, g0):
    sAB = m0 * m0
    smin, smax, p, q = pdg_line(sAB, ch, DZ)
    s12, s13 = to_s12_s13(ch, sAB, 0.5 * (smin + smax), DZ)
    for J in (0, 1, 2):
        r = oracle_mod.res_amp(DZ, ch, m0, g0, J, s12, s13)
        assert abs(r["width"] - g0) < 1e-14
        assert abs(r["B"] - 1.0) < 1e-14
        assert abs(abs(r["BW"]) ** 2 - 1 / (m0 * g0) ** 2) < 1e-12 / (m0 * g0) ** 2
    # off the pole: Im BW = m0 Gamma(s) |BW|^2
    s12, s13 = to_s12_s13(ch, sAB * 1.07, None, DZ) if False else (s12, s13)
    for sab in (0.9 * sAB, 1.1 * sAB):
        lo_, hi_, _, _ = pdg_line(sab, ch, DZ)
        a, b = to_s12_s13(ch, sab, 0.5 * (lo_ + hi_), DZ)
        r = oracle_mod.res_amp(DZ, ch, m0, g0, 1, a, b)
        assert abs(r["BW"].imag - m0 * r["width"] * abs(r["BW"]) ** 2) < 1e-13 * abs(r["BW"].imag)


@pytest.mark.parametrize("ch", ["23", "12", "13"])
def test_zemach_factors_are_legendre(oracle_mod, ch):
    """Along a fixed-s_AB line Z_J is (4pq)^J times P_1 / (2/3) P_2 of
    cos(theta) (linear in s_AC): ends of Z_1 = +-4pq, of Z_2 = 2/3 (4pq)^2,
    and Z_0, Z_1, Z_2 are mutually orthogonal over the line."""
    sAB = 1.1 if ch != "23" else 0.8
    smin, smax, p, q = pdg_line(sAB, ch, DZ)

    def Z(J, sAC):
        a, b = to_s12_s13(ch, sAB, sAC, DZ)
        return oracle_mod.res_amp(DZ, ch, 1.0, 0.1, J, a, b)["Z"]

    k = 4 * p * q
    assert abs(abs(Z(1, smin)) - k) < 1e-11 * k and abs(abs(Z(1, smax)) - k) < 1e-11 * k
    assert Z(1, smin) * Z(1, smax) < 0
    for s in (smin, smax):
        assert abs(Z(2, s) - 2.0 / 3.0 * k * k) < 1e-11 * k * k
    for J1, J2 in ((0, 1), (0, 2), (1, 2)):
        v = integrate.quad(lambda s: Z(J1, s) * Z(J2, s), smin, smax, epsabs=1e-14, limit=200)[0]
        norm = math.sqrt(integrate.quad(lambda s: Z(J1, s) ** 2, smin, smax)[0] *
                         integrate.quad(lambda s: Z(J2, s) ** 2, smin, smax)[0])
        assert abs(v) < 1e-12 * norm


def test_pipi_spin_factor_symmetry(oracle_mod):
    """For a pi pi resonance the 2 <-> 3 swap flips Z_1 and keeps Z_2."""
    for s12, s13 in ((1.0, 1.2), (0.9, 1.6), (1.4, 1.3)):
        if not oracle_mod.inside(DZ, s12, s13):
            continue
        z1 = oracle_mod.res_amp(DZ, "23", 0.775, 0.149, 1, s12, s13)["Z"]
        z1s = oracle_mod.res_amp(DZ, "23", 0.775, 0.149, 1, s13, s12)["Z"]
        z2 = oracle_mod.res_amp(DZ, "23", 1.275, 0.185, 2, s12, s13)["Z"]
        z2s = oracle_mod.res_amp(DZ, "23", 1.275, 0.185, 2, s13, s12)["Z"]
        assert abs(z1 + z1s) < 1e-13 and abs(z2 - z2s) < 1e-13


def grid_cells(dz):
    lo, hi = S.dalitz_box(dz)
    G = dz["grid"]
    h = (hi - lo) / G
    c = lo + (np.arange(G) + 0.5) * h
    a, b = np.meshgrid(c, c, indexing="ij")
    return a.ravel(), b.ravel(), h * h


def test_dalitz_grid_matrices_brute_force(oracle_mod):
    """I, Ibar and J against a brute-force sum of |A|^2, |Abar|^2 and
    Re(conj(A) Abar) over the grid cells (a separate code path)."""
    m = oracle_mod.Model(S.C4)
    th = m.theta(S.C4["truth"])
    a, b, area = grid_cells(DZ)
    A2 = m.dalitz_amp2(th, a, b)
    B2 = m.dalitz_amp2(th, a, b, swapped=True)
    X = m.dalitz_cross(th, a, b)
    c = np.array([1.0 + 0j] + [complex(th[2 * k], th[2 * k + 1]) for k in range(8)])
    I, Ib, J = m.dalitz_matrix(0), m.dalitz_matrix(1), m.dalitz_matrix(2)
    assert abs((c.conj() @ I @ c).real - math.fsum(A2) * area) < 1e-12 * math.fsum(A2) * area
    assert abs((c.conj() @ Ib @ c).real - math.fsum(B2) * area) < 1e-12 * math.fsum(B2) * area
    assert abs((c.conj() @ J @ c).real - math.fsum(X) * area) < 1e-11 * math.fsum(A2) * area
    assert np.abs(I - I.conj().T).max() == 0.0
    assert np.abs(I - Ib).max() < 1e-13 * np.abs(I).max()   # symmetric grid
    # c = 0: uniform density 1 / (grid area)
    m3 = oracle_mod.Model(S.C3)
    z = np.zeros(16)
    lp = m3.logpdf(z, {"s12": a[A2 > 0][:50], "s13": b[A2 > 0][:50]})
    assert np.allclose(lp, -math.log(I[0, 0].real), atol=1e-14, rtol=0)


def test_dalitz_norm_converges_with_grid(oracle_mod):
    import copy
    th = None
    vals = []
    for G in (500, 1000, 2000):
        spec = copy.deepcopy(S.C3)
        spec["model"]["dalitz"]["grid"] = G
        m = oracle_mod.Model(spec)
        th = m.theta(S.C3["truth"])
        vals.append(math.exp(m.node_lnnorm(m.root, th)[0]))
    assert abs(vals[2] - vals[1]) < 0.5 * abs(vals[1] - vals[0]) + 1e-6 * vals[2]
    assert abs(vals[2] - vals[1]) < 2e-4 * vals[2]


def test_tddp_time_integral_and_y0_factorisation(oracle_mod):
    m4 = oracle_mod.Model(S.C4)
    m3 = oracle_mod.Model(S.C3)
    th4 = m4.theta(S.C4["truth"])
    tau, y = th4[-2], th4[-1]
    pts = [(1.0, 1.2), (0.7, 2.0), (1.8, 0.9)]
    lnNT = m4.node_lnnorm(m4.root, th4)[0]
    for s12, s13 in pts:
        a2 = m4.dalitz_amp2(th4, [s12], [s13])[0]
        b2 = m4.dalitz_amp2(th4, [s12], [s13], swapped=True)[0]
        x = m4.dalitz_cross(th4, [s12], [s13])[0]
        for st in (0.02, 0.2):
            f = lambda t: math.exp(m4.logpdf(th4, {"s12": np.array([s12]), "s13": np.array([s13]),
                                                   "t": np.array([t]), "sigma_t": np.array([st])})[0] + lnNT)
            val = integrate.quad(f, -3.0, 15.0, points=[0.0], epsabs=0, epsrel=1e-12, limit=400)[0]
            ac, a0, as_ = 0.5 * (a2 + b2), 0.5 * (a2 - b2), -x
            ref = ac * tau / (1 - y * y) + a0 * tau + as_ * y * tau / (1 - y * y)
            assert abs(val - ref) < 1e-10 * ref
    # y = 0: P_tddp = P_dalitz * (1/tau) E(t; 1/tau, sigma_t)
    th0 = th4.copy()
    th0[-1] = 0.0
    rng = np.random.default_rng(2)
    ev = {"s12": np.array([1.0, 0.7, 1.8]), "s13": np.array([1.2, 2.0, 0.9]),
          "t": rng.uniform(-0.2, 2, 3), "sigma_t": rng.uniform(0.02, 0.2, 3)}
    lp4 = m4.logpdf(th0, ev)
    lp3 = m3.logpdf(th0[:-2], ev)
    e = np.array([oracle_mod.econv(t, 1 / tau, s) for t, s in zip(ev["t"], ev["sigma_t"])])
    assert np.allclose(lp4, lp3 + np.log(e / tau), atol=1e-12, rtol=0)


def test_tddp_density_positive_on_scan(oracle_mod):
    m4 = oracle_mod.Model(S.C4)
    th = m4.theta(S.C4["truth"])
    for y in (-0.2, 0.01, 0.2):
        th[-1] = y
        a, b, _ = grid_cells(dict(DZ, grid=60))
        keep = m4.dalitz_amp2(th, a, b) > 0
        a, b = a[keep], b[keep]
        for t in (-0.5, 0.0, 0.4, 2.0, 6.0):
            for st in (0.02, 0.2):
                lp = m4.logpdf(th, {"s12": a, "s13": b, "t": np.full(a.size, t),
                                    "sigma_t": np.full(a.size, st)})
                assert np.all(np.isfinite(lp))


@pytest.mark.parametrize("cfg", ["c3", "c4"])
def test_dalitz_gradients_match_finite_differences(oracle_mod, cfg):
    spec = S.workload(cfg)
    m = oracle_mod.Model(spec)
    th = m.theta(spec["truth"])
    rng = np.random.default_rng(5)
    a, b, _ = grid_cells(dict(DZ, grid=80))
    keep = m.dalitz_amp2(th, a, b) > 0
    n = 400
    idx = rng.choice(np.nonzero(keep)[0], n, replace=False)
    d = {"s12": a[idx], "s13": b[idx]}
    if cfg == "c4":
        d["sigma_t"] = rng.uniform(0.02, 0.2, n)
        d["t"] = rng.exponential(0.41, n) + d["sigma_t"] * rng.standard_normal(n)
    th = th * (1 + 0.05 * rng.standard_normal(th.size))
    v, g = m.nll(th, d, grad=True)
    gf = fd_grad(m, th, d, rel=1e-6)
    scale = np.abs(m.logpdf(th, d, grad_rows=True)[1]).sum(axis=0)
    assert np.all(np.abs(g - gf) <= 1e-7 * scale + 1e-7)
