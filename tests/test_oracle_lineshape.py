"""Pins of the oracle's resonance lineshape away from the pole.

At s = m0^2 the mass-dependent width equals Gamma0 and the barrier ratio 1
whatever the formula, so the pole alone cannot catch a wrong exponent of
q/q0, a barrier factor taken once instead of squared in the width, or a
missing m0/sqrt(s).  These tests fix the lineshape by properties that do
not restate the oracle's formula:

* the threshold law: Gamma(s) ~ q^(2J+1) as q -> 0 (the centrifugal
  barrier of a spin-J decay);
* the barrier-damped limit: Gamma(s) sqrt(s) ~ q as q -> infinity for every
  J (the Blatt-Weisskopf factors cancel the centrifugal growth);
* the absolute value off the pole against the width written in the
  von Hippel-Quigg form Gamma0 (q/q0) (m0/sqrt s) F_J^2(q) / F_J^2(q0), with
  F_J the normalised Blatt-Weisskopf penetration factors
  (F_1^2 = 2z/(1+z), F_2^2 = 13z^2/((z-3)^2 + 9z), z = (qr)^2), the
  momentum from the two-body formula in 40-digit arithmetic, and the
  relativistic Breit-Wigner 1/(m0^2 - s - i m0 Gamma(s)) built from it.

The amplitude convention is that of the coherent sum of the paper's Dalitz
fit (section "Results"); the width law is the standard mass-dependent one.
"""
import math

import mpmath as mp
import pytest

import synthgen as S

DZ = S.C3["model"]["dalitz"]
R = DZ["r"]


def masses(ch):
    """(m_A, m_B, m_C) of the resonance's daughters and the bachelor."""
    return {"23": (DZ["m2"], DZ["m3"], DZ["m1"]), "12": (DZ["m1"], DZ["m2"], DZ["m3"]),
            "13": (DZ["m1"], DZ["m3"], DZ["m2"])}[ch]


def s_of_q(ch, q):
    """Invariant mass squared of the pair whose daughters have momentum q in
    its rest frame."""
    mA, mB, _ = masses(ch)
    return (math.sqrt(mA * mA + q * q) + math.sqrt(mB * mB + q * q)) ** 2


def point(ch, sAB):
    """(s12, s13) with the channel's pair at sAB (the other invariant is
    arbitrary: the width and barrier do not depend on it)."""
    tot = DZ["M"] ** 2 + DZ["m1"] ** 2 + DZ["m2"] ** 2 + DZ["m3"] ** 2
    if ch == "23":
        s12 = 1.0
        return s12, tot - sAB - s12
    if ch == "12":
        return sAB, 1.0
    return 1.0, sAB


def width(oracle_mod, ch, m0, g0, J, sAB):
    a, b = point(ch, sAB)
    return oracle_mod.res_amp(DZ, ch, m0, g0, J, a, b)


# (channel, m0, Gamma0): a resonance in each pair of the three-body decay
RES = [("23", 0.775, 0.149), ("12", 0.892, 0.05), ("13", 1.1, 0.2)]


@pytest.mark.parametrize("ch,m0,g0", RES)
@pytest.mark.parametrize("J", [0, 1, 2])
def test_threshold_law(oracle_mod, ch, m0, g0, J):
    """d ln Gamma / d ln q -> 2J + 1 at threshold; a q/q0 exponent of 2J or
    2J + 2 gives a slope off by one."""
    q1, q2 = 1e-4, 2e-4
    w1 = width(oracle_mod, ch, m0, g0, J, s_of_q(ch, q1))["width"]
    w2 = width(oracle_mod, ch, m0, g0, J, s_of_q(ch, q2))["width"]
    slope = math.log(w2 / w1) / math.log(q2 / q1)
    assert abs(slope - (2 * J + 1)) < 1e-4, slope


@pytest.mark.parametrize("ch,m0,g0", RES)
@pytest.mark.parametrize("J", [0, 1, 2])
def test_barrier_damped_limit(oracle_mod, ch, m0, g0, J):
    """d ln(Gamma sqrt s) / d ln q -> 1 for large q and every J: the squared
    barrier ratio cancels q^(2J).  A barrier factor taken once in the width
    gives slope J + 1, a missing m0/sqrt(s) adds one."""
    q1, q2 = 40.0, 80.0
    s1, s2 = s_of_q(ch, q1), s_of_q(ch, q2)
    w1 = width(oracle_mod, ch, m0, g0, J, s1)["width"] * math.sqrt(s1)
    w2 = width(oracle_mod, ch, m0, g0, J, s2)["width"] * math.sqrt(s2)
    slope = math.log(w2 / w1) / math.log(q2 / q1)
    # corrections are O(1 / (q r)^2) < 2e-3
    assert abs(slope - 1.0) < 3e-3, slope


def hippel_quigg_F2(J, z):
    if J == 0:
        return mp.mpf(1)
    if J == 1:
        return 2 * z / (1 + z)
    return 13 * z * z / ((z - 3) ** 2 + 9 * z)


def momentum(ch, s):
    mA, mB, _ = masses(ch)
    mA, mB = mp.mpf(mA), mp.mpf(mB)
    return mp.sqrt((s - (mA + mB) ** 2) * (s - (mA - mB) ** 2)) / (2 * mp.sqrt(s))


@pytest.mark.parametrize("ch,m0,g0", RES)
@pytest.mark.parametrize("J", [0, 1, 2])
def test_lineshape_off_pole(oracle_mod, ch, m0, g0, J):
    """Gamma(s), B_J(q) and the Breit-Wigner at points across the pair's
    physical range against the von Hippel-Quigg form, 1e-12 relative."""
    mp.mp.dps = 40
    mA, mB, mC = masses(ch)
    s_lo, s_hi = (mA + mB) ** 2, (DZ["M"] - mC) ** 2
    m0m = mp.mpf(m0)
    q0 = momentum(ch, m0m * m0m)
    z0 = (q0 * R) ** 2
    for frac in (0.02, 0.1, 0.3, 0.45, 0.6, 0.8, 0.97):
        s = s_lo + frac * (s_hi - s_lo)
        r = width(oracle_mod, ch, m0, g0, J, s)
        sm = mp.mpf(s)
        q = momentum(ch, sm)
        z = (q * R) ** 2
        gam = g0 * (q / q0) * (m0m / mp.sqrt(sm)) * hippel_quigg_F2(J, z) / hippel_quigg_F2(J, z0)
        barrier = mp.sqrt(hippel_quigg_F2(J, z) / hippel_quigg_F2(J, z0)) * (q0 / q) ** J
        bw = 1 / mp.mpc(m0m * m0m - sm, -m0m * gam)
        assert abs(r["width"] - float(gam)) <= 1e-12 * float(gam), (frac, r["width"], gam)
        assert abs(r["B"] - float(barrier)) <= 1e-12 * float(barrier), (frac, r["B"], barrier)
        assert abs(r["BW"] - complex(bw)) <= 1e-12 * abs(complex(bw)), (frac, r["BW"], bw)
        amp = complex(bw) * float(barrier) * r["Z"]
        assert abs(r["A"] - amp) <= 1e-12 * max(abs(amp), 1e-300), (frac, r["A"], amp)
