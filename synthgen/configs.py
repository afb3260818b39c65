"""Workload descriptions: observables, parameters, model trees and sizes.

Everything here is plain data.  A model tree is a nested dict:

  {"op": "exp",    "obs": "x", "par": ["alpha"]}
  {"op": "gauss",  "obs": "x", "par": ["mu", "sigma"]}
  {"op": "poly",   "obs": "x", "par": ["a1", ...], "x0": 0.0}
  {"op": "add",    "par": ["f1", ...], "children": [...]}   # K children, K-1 fractions
  {"op": "prod",   "children": [...]}
  {"op": "dalitz", "obs": ["s12", "s13"], "par": [re1, im1, re2, im2, ...],
                   "dalitz": DALITZ_KINEMATICS}
  {"op": "tddp",   "obs": ["s12", "s13", "t", "sigma_t"],
                   "par": [re1, im1, ..., "tau", "y"], "dalitz": DALITZ_KINEMATICS}
  full time-dependent model: "x": True / "qp": True on the tddp node and
  "float": True on resonances; "par" then lists 2R coefficients, tau, y,
  (x), (|q/p|, arg q/p), then (m0, Gamma0) of each floating resonance

Observables are (name, lo, hi); parameters are (name, init, step, lo, hi,
fixed) as in the two Variable constructors of the paper's first listing.
Unbounded parameters use lo = hi = 0.
"""
import math

__all__ = [
    "C1", "C2", "C3", "C4", "C4X", "C5", "LISTING2", "MAPPED", "MAPPED_SUM", "SHARED", "SHARED_SUM",
    "SHARED_2D", "C4S", "C4F", "CONV", "CONV_POLY", "CONV_GMIX", "COMP", "RESONANCES_FULL", "SIGMA_T_CELLS", "SIGMA_T_BOUNDS", "DALITZ_KINEMATICS", "RESONANCES",
    "DALITZ_TRUTH", "dalitz_param_names", "dalitz_box", "workload",
]

# ---------------------------------------------------------------- C1
# 1-D exponential e^{alpha x} on [0, 10]; the paper's first listing uses
# start -2, step 0.1 and bounds [-10, 10] for alpha.
C1 = {
    "name": "c1_exp",
    "obs": [("x", 0.0, 10.0)],
    "params": [("alpha", -2.0, 0.1, -10.0, 10.0, False)],
    "truth": {"alpha": -0.5},
    "model": {"op": "exp", "obs": "x", "par": ["alpha"]},
    "n_events": 100_000,
    "seed": 1,
}

# ---------------------------------------------------------------- C2
# f * Gauss(x; mu, sigma) + (1 - f) * exp(beta x) on [5.2, 5.3].
C2 = {
    "name": "c2_gauss_exp",
    "obs": [("x", 5.2, 5.3)],
    "params": [
        ("f", 0.25, 0.01, 0.0, 1.0, False),
        ("mu", 5.279, 0.001, 5.2, 5.3, False),
        ("sigma", 0.0035, 0.0005, 1e-4, 0.05, False),
        ("beta", -1.5, 0.1, -10.0, 10.0, False),
    ],
    "truth": {"f": 0.3, "mu": 5.28, "sigma": 0.003, "beta": -2.0},
    "model": {
        "op": "add", "par": ["f"],
        "children": [
            {"op": "gauss", "obs": "x", "par": ["mu", "sigma"]},
            {"op": "exp", "obs": "x", "par": ["beta"]},
        ],
    },
    "n_events": 10_000_000,
    "seed": 2,
}

# ---------------------------------------------------------------- Dalitz
# Parent of 1.865 GeV into K_S (1), pi+ (2), pi- (3); Blatt-Weisskopf radius
# 1.5 / GeV; normalisation on a 1000 x 1000 midpoint grid.
DALITZ_KINEMATICS = {
    "M": 1.865, "m1": 0.4976, "m2": 0.1396, "m3": 0.1396,
    "r": 1.5, "grid": 1000,
}

# Eight relativistic Breit-Wigner resonances: (channel, m0, Gamma0, J).
# Channel "23" is pi+ pi-, "12" is K_S pi+, "13" is K_S pi-.
RESONANCES = [
    ("23", 0.500, 0.400, 0),
    ("23", 0.775, 0.149, 1),
    ("23", 0.783, 0.010, 1),
    ("23", 1.275, 0.185, 2),
    ("12", 0.892, 0.050, 1),
    ("13", 0.892, 0.050, 1),
    ("12", 1.425, 0.270, 0),
    ("12", 1.717, 0.322, 1),
]

# True complex coefficients c_1..c_8 (the non-resonant c_0 is fixed to 1).
DALITZ_TRUTH = [
    (0.343812, 0.198500), (0.277, 0.0), (-0.005233, 0.014377),
    (0.339229, -0.123469), (-0.297225, 0.249402), (0.047035, -0.039467),
    (0.353500, 0.612280), (-0.232689, -1.319642),
]


def dalitz_param_names(n_res=len(RESONANCES)):
    out = []
    for k in range(1, n_res + 1):
        out += [f"re{k}", f"im{k}"]
    return out


def dalitz_box(kin=DALITZ_KINEMATICS):
    """Bounding box [(m1+m2)^2, (M-m3)^2] of s12 (and, for m2 = m3, of s13)."""
    lo = (kin["m1"] + kin["m2"]) ** 2
    hi = (kin["M"] - kin["m3"]) ** 2
    return lo, hi


def _dalitz_start(seed=7):
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for re, im in DALITZ_TRUTH:
        mag = math.hypot(re, im) * (1.0 + 0.1 * rng.standard_normal())
        ph = math.atan2(im, re) + math.radians(10.0) * rng.standard_normal()
        out.append((mag * math.cos(ph), mag * math.sin(ph)))
    return out


def _dalitz_params(start):
    ps = []
    for k, (re, im) in enumerate(start, start=1):
        ps.append((f"re{k}", re, 0.05, 0.0, 0.0, False))
        ps.append((f"im{k}", im, 0.05, 0.0, 0.0, False))
    return ps


_BOX = dalitz_box()
_RES_SPEC = [{"ch": ch, "m0": m0, "g0": g0, "J": J} for ch, m0, g0, J in RESONANCES]

C3 = {
    "name": "c3_dalitz",
    "obs": [("s12", _BOX[0], _BOX[1]), ("s13", _BOX[0], _BOX[1])],
    "params": _dalitz_params(_dalitz_start()),
    "truth": {n: v for n, v in zip(dalitz_param_names(), [c for p in DALITZ_TRUTH for c in p])},
    "model": {
        "op": "dalitz", "obs": ["s12", "s13"], "par": dalitz_param_names(),
        "dalitz": dict(DALITZ_KINEMATICS, resonances=_RES_SPEC),
    },
    "n_events": 1_000_000,
    "seed": 3,
}

# ---------------------------------------------------------------- C4
# Decay time with per-event Gaussian resolution times the C3 amplitude.
# t and sigma_t are conditioning observables with no finite normalisation box
# (t is normalised over the real line); the declared ranges only bound the
# values a dataset may hold.
C4 = {
    "name": "c4_tddp",
    "obs": [("s12", _BOX[0], _BOX[1]), ("s13", _BOX[0], _BOX[1]),
            ("t", -math.inf, math.inf), ("sigma_t", 0.0, math.inf)],
    "params": _dalitz_params(_dalitz_start()) + [
        ("tau", 0.45, 0.01, 0.1, 2.0, False),
        ("y", 0.0, 0.005, -0.2, 0.2, False),
    ],
    "truth": dict(C3["truth"], tau=0.41, y=0.01),
    "model": {
        "op": "tddp", "obs": ["s12", "s13", "t", "sigma_t"],
        "par": dalitz_param_names() + ["tau", "y"],
        "dalitz": dict(DALITZ_KINEMATICS, resonances=_RES_SPEC),
    },
    "sigma_t_range": (0.02, 0.2),
    "n_events": 2_000_000,
    "seed": 4,
}

# ---------------------------------------------------------------- C4X
# C4 with the mixing parameter x free as well: the trigonometric time terms
# (cos / sin (x t / tau) convolved with the resolution) join the hyperbolic
# ones.  The parameter vector ends tau, y, x.
C4X = {
    "name": "c4x_tddp_mixing",
    "obs": C4["obs"],
    "params": C4["params"] + [("x", 0.0, 0.005, -0.2, 0.2, False)],
    "truth": dict(C4["truth"], x=0.008),
    "model": {
        "op": "tddp", "obs": ["s12", "s13", "t", "sigma_t"],
        "par": dalitz_param_names() + ["tau", "y", "x"],
        "dalitz": dict(DALITZ_KINEMATICS, resonances=_RES_SPEC),
    },
    "sigma_t_range": C4["sigma_t_range"],
    "n_events": 2_000_000,
    "seed": 6,
}

# ---------------------------------------------------------------- C4F
# The full mixing model of the paper's time-dependent fit: 16 complex
# amplitudes (the non-resonant term and 15 resonances), decay time with x
# and y, complex q/p = |q/p| e^{i phi}, and the masses and widths of the
# rho(770) and of the K*(892) in the 12 pair as parameters (their
# normalisation is then re-computed on the grid at every evaluation):
# 30 + 3 + 2 + 4 = 39 parameters.  Coefficients: magnitudes chosen for the
# fit fractions (NR .058, then .093 .232 .006 .035 .023 .023 .012 .463 .012
# .070 .012 .012 .006 .035 .012 on the 400 x 400 grid), phases (30, 0, 110,
# -60, -20, 80, 150, 140, -40, 60, -100, 20, -150, 100, 45) degrees.
RESONANCES_FULL = [
    ("23", 0.500, 0.400, 0), ("23", 0.775, 0.149, 1), ("23", 0.783, 0.010, 1), ("23", 0.980, 0.060, 0),
    ("23", 1.275, 0.185, 2), ("23", 1.370, 0.350, 0), ("23", 1.465, 0.400, 1),
    ("12", 0.892, 0.050, 1), ("13", 0.892, 0.050, 1), ("12", 1.425, 0.270, 0), ("13", 1.425, 0.270, 0),
    ("12", 1.430, 0.100, 2), ("13", 1.430, 0.100, 2), ("12", 1.717, 0.322, 1), ("13", 1.414, 0.232, 1),
]
FULL_TRUTH = [
    (0.389105, 0.224650), (0.349743, 0.0), (-0.004659, 0.012801), (0.068723, -0.119032),
    (0.350606, -0.127610), (0.105086, 0.595975), (-0.370700, 0.214024), (-0.376222, 0.315688),
    (0.059486, -0.049915), (0.346499, 0.600155), (-0.049128, -0.278617), (0.296423, 0.107889),
    (-0.193171, -0.111527), (-0.192947, 1.094255), (0.214472, 0.214472),
]
FULL_FLOATING = {1: ("rho_m0", "rho_g0", (0.70, 0.85), (0.10, 0.20)),
                 7: ("kst_m0", "kst_g0", (0.85, 0.93), (0.03, 0.08))}


def _full_model(grid=1000, n_events=1_000_000, seed=8):
    import numpy as np
    rng = np.random.default_rng(seed + 100)
    R = len(RESONANCES_FULL)
    res, shape_par, shape_names, truth = [], [], [], {}
    for k, (ch, m0, g0, J) in enumerate(RESONANCES_FULL):
        r = {"ch": ch, "m0": m0, "g0": g0, "J": J}
        if k in FULL_FLOATING:
            nm, ng, bm, bg = FULL_FLOATING[k]
            r["float"] = True
            shape_par += [(nm, m0 * (1.0 + 0.01 * rng.standard_normal()), 0.002, bm[0], bm[1], False),
                          (ng, g0 * (1.0 + 0.05 * rng.standard_normal()), 0.002, bg[0], bg[1], False)]
            shape_names += [nm, ng]
            truth[nm], truth[ng] = m0, g0
        res.append(r)
    coef = []
    for k, (re, im) in enumerate(FULL_TRUTH, start=1):
        mag = math.hypot(re, im) * (1.0 + 0.1 * rng.standard_normal())
        ph = math.atan2(im, re) + math.radians(10.0) * rng.standard_normal()
        coef += [(f"re{k}", mag * math.cos(ph), 0.05, 0.0, 0.0, False),
                 (f"im{k}", mag * math.sin(ph), 0.05, 0.0, 0.0, False)]
        truth[f"re{k}"], truth[f"im{k}"] = re, im
    params = coef + [("tau", 0.45, 0.01, 0.1, 2.0, False), ("y", 0.0, 0.005, -0.2, 0.2, False),
                     ("x", 0.0, 0.005, -0.2, 0.2, False), ("qp_mag", 1.05, 0.02, 0.5, 1.5, False),
                     ("qp_phase", 0.05, 0.02, -1.0, 1.0, False)] + shape_par
    truth.update(tau=0.41, y=0.01, x=0.008, qp_mag=1.0, qp_phase=0.0)
    box = dalitz_box()
    return {
        "name": "c4f_tddp_full_mixing",
        "obs": [("s12", box[0], box[1]), ("s13", box[0], box[1]),
                ("t", -math.inf, math.inf), ("sigma_t", 0.0, math.inf)],
        "params": params,
        "truth": truth,
        "model": {
            "op": "tddp", "obs": ["s12", "s13", "t", "sigma_t"], "x": True, "qp": True,
            "par": dalitz_param_names(R) + ["tau", "y", "x", "qp_mag", "qp_phase"] + shape_names,
            "dalitz": dict(DALITZ_KINEMATICS, grid=grid, resonances=res),
        },
        "sigma_t_range": (0.02, 0.2),
        "n_events": n_events,
        "seed": seed,
    }


C4F = _full_model()

# ---------------------------------------------------------------- mapped densities
# The MappedPdf form of section "Combining functions": a different leaf on
# each of three ranges of x (exponential on [0, 4), Gaussian on [4, 7),
# quadratic on [7, 10]); and the same map added to an exponential
# background (the map then normalised per event inside the sum).
MAPPED = {
    "name": "mapped3",
    "obs": [("x", 0.0, 10.0)],
    "params": [("m_alpha", -0.25, 0.05, -5.0, 5.0, False), ("m_mu", 5.4, 0.05, 3.0, 8.0, False),
               ("m_sigma", 0.7, 0.05, 0.05, 5.0, False), ("m_a1", 0.12, 0.02, 0.0, 0.0, False),
               ("m_a2", 0.012, 0.002, 0.0, 0.0, False)],
    "truth": {"m_alpha": -0.3, "m_mu": 5.5, "m_sigma": 0.6, "m_a1": 0.1, "m_a2": 0.01},
    "model": {"op": "map", "obs": "x", "bounds": [4.0, 7.0], "children": [
        {"op": "exp", "obs": "x", "par": ["m_alpha"]},
        {"op": "gauss", "obs": "x", "par": ["m_mu", "m_sigma"]},
        {"op": "poly", "obs": "x", "par": ["m_a1", "m_a2"], "x0": 8.5},
    ]},
    "n_events": 10_000_000,
    "seed": 21,
}
MAPPED_SUM = {
    "name": "mapped3_plus_exp",
    "obs": [("x", 0.0, 10.0)],
    "params": MAPPED["params"] + [("m_f", 0.6, 0.05, 0.0, 1.0, False), ("m_beta", -0.1, 0.05, -5.0, 5.0, False)],
    "truth": dict(MAPPED["truth"], m_f=0.7, m_beta=-0.15),
    "model": {"op": "add", "par": ["m_f"], "children": [
        MAPPED["model"], {"op": "exp", "obs": "x", "par": ["m_beta"]}]},
    "n_events": 10_000_000,
    "seed": 22,
}

# ---------------------------------------------------------------- products over a shared observable
# An acceptance (quadratic in x) times a Gaussian signal on the same x: the
# product is renormalised numerically (section "Combining functions":
# ProdPdf); the same product added to an exponential background; and the
# product times an independent exponential in y.
SHARED = {
    "name": "acceptance_x_gauss",
    "obs": [("x", 0.0, 10.0)],
    "params": [("e_a1", 0.04, 0.02, 0.0, 0.0, False), ("e_a2", -0.008, 0.005, 0.0, 0.0, False),
               ("s_mu", 6.2, 0.1, 0.0, 10.0, False), ("s_sigma", 1.1, 0.1, 0.05, 5.0, False)],
    "truth": {"e_a1": 0.05, "e_a2": -0.01, "s_mu": 6.0, "s_sigma": 1.2},
    "model": {"op": "prod", "children": [
        {"op": "poly", "obs": "x", "par": ["e_a1", "e_a2"], "x0": 5.0},
        {"op": "gauss", "obs": "x", "par": ["s_mu", "s_sigma"]},
    ]},
    "n_events": 10_000_000,
    "seed": 23,
}
SHARED_SUM = {
    "name": "acceptance_x_gauss_plus_exp",
    "obs": [("x", 0.0, 10.0)],
    "params": SHARED["params"] + [("s_f", 0.6, 0.05, 0.0, 1.0, False), ("b_beta", -0.2, 0.05, -5.0, 5.0, False)],
    "truth": dict(SHARED["truth"], s_f=0.55, b_beta=-0.25),
    "model": {"op": "add", "par": ["s_f"], "children": [
        SHARED["model"], {"op": "exp", "obs": "x", "par": ["b_beta"]}]},
    "n_events": 10_000_000,
    "seed": 24,
}
SHARED_2D = {
    "name": "acceptance_x_gauss_times_exp_y",
    "obs": [("x", 0.0, 10.0), ("y", 0.0, 5.0)],
    "params": SHARED["params"] + [("y_alpha", -0.4, 0.05, -5.0, 5.0, False)],
    "truth": dict(SHARED["truth"], y_alpha=-0.5),
    "model": {"op": "prod", "children": SHARED["model"]["children"] + [
        {"op": "exp", "obs": "y", "par": ["y_alpha"]}]},
    "n_events": 1_000_000,
    "seed": 25,
}

# ---------------------------------------------------------------- C4S
# C4 with a density for the decay-time uncertainty that varies across the
# Dalitz plot: the plot's box is cut at s12 = 1.5 and s13 = 1.5 GeV^2 into a
# 2 x 2 grid of cells, each with a Gaussian sigma_t density on [0.02, 0.2] ps
# (cells row-major, s12 index first); the model is the product of the
# time-dependent density (conditional on sigma_t) and that map.
SIGMA_T_CELLS = [(0.08, 0.03), (0.10, 0.035), (0.12, 0.04), (0.14, 0.045)]
SIGMA_T_BOUNDS = ([1.5], [1.5])
C4S = {
    "name": "c4s_tddp_sigma_t_map",
    "obs": [("s12", _BOX[0], _BOX[1]), ("s13", _BOX[0], _BOX[1]),
            ("t", -math.inf, math.inf), ("sigma_t", 0.02, 0.2)],
    "params": C4["params"] + [p for c in range(4) for p in (
        (f"st_mu{c}", 0.11, 0.005, 0.0, 0.5, False), (f"st_sg{c}", 0.05, 0.005, 0.005, 0.5, False))],
    "truth": dict(C4["truth"], **{k: v for c, (mu, sg) in enumerate(SIGMA_T_CELLS)
                                  for k, v in ((f"st_mu{c}", mu), (f"st_sg{c}", sg))}),
    "model": {"op": "prod", "children": [
        C4["model"],
        {"op": "dpmap", "obs": ["s12", "s13", "sigma_t"], "b12": SIGMA_T_BOUNDS[0], "b13": SIGMA_T_BOUNDS[1],
         "children": [{"op": "gauss", "obs": "sigma_t", "par": [f"st_mu{c}", f"st_sg{c}"]} for c in range(4)]},
    ]},
    "sigma_t_range": (0.02, 0.2),
    "n_events": 2_000_000,
    "seed": 7,
}

# ---------------------------------------------------------------- CONV
# Numerical convolution (ConvolutionPdf): an exponential model smeared by a
# Gaussian resolution (residual range [-2, 2], 400 grid points), plus an
# exponential background; and a quadratic model smeared by a one-sided
# exponential resolution on [0, 1].
CONV = {
    "name": "conv_exp_gauss_plus_exp",
    "obs": [("x", 0.0, 10.0)],
    "params": [("c_alpha", -0.3, 0.05, -5.0, 5.0, False), ("r_mu", 0.0, 0.02, -1.0, 1.0, False),
               ("r_sigma", 0.4, 0.02, 0.02, 2.0, False), ("c_f", 0.6, 0.05, 0.0, 1.0, False),
               ("b_beta", -0.05, 0.02, -5.0, 5.0, False)],
    "truth": {"c_alpha": -0.4, "r_mu": 0.05, "r_sigma": 0.3, "c_f": 0.7, "b_beta": -0.1},
    "model": {"op": "add", "par": ["c_f"], "children": [
        {"op": "conv", "obs": "x", "grid": 400, "d_lo": -2.0, "d_hi": 2.0, "children": [
            {"op": "exp", "obs": "x", "par": ["c_alpha"]},
            {"op": "gauss", "obs": "x", "par": ["r_mu", "r_sigma"]}]},
        {"op": "exp", "obs": "x", "par": ["b_beta"]}]},
    "n_events": 1_000_000,
    "seed": 26,
}
CONV_POLY = {
    "name": "conv_poly_onesided",
    "obs": [("x", 0.0, 10.0)],
    "params": [("p_a1", 0.05, 0.02, 0.0, 0.0, False), ("p_a2", -0.01, 0.005, 0.0, 0.0, False),
               ("r_alpha", -3.0, 0.2, -20.0, -0.1, False)],
    "truth": {"p_a1": 0.1, "p_a2": -0.02, "r_alpha": -4.0},
    "model": {"op": "conv", "obs": "x", "grid": 256, "d_lo": 0.0, "d_hi": 1.0, "children": [
        {"op": "poly", "obs": "x", "par": ["p_a1", "p_a2"], "x0": 5.0},
        {"op": "exp", "obs": "x", "par": ["r_alpha"]}]},
    "n_events": 1_000_000,
    "seed": 27,
}

# Nested composition: the exponential smeared by a resolution made of two
# Gaussians (a core and a wider tail, each normalised over the residual
# range), plus an exponential background -- the shape of the paper's binned
# example, a lineshape convolved with a resolution of several Gaussians.
CONV_GMIX = {
    "name": "conv_exp_gaussmix_plus_exp",
    "obs": [("x", 0.0, 10.0)],
    "params": [("c_alpha", -0.3, 0.05, -5.0, 5.0, False), ("r_mu1", 0.0, 0.02, -1.0, 1.0, False),
               ("r_sg1", 0.25, 0.02, 0.02, 2.0, False), ("r_mu2", 0.0, 0.02, -1.0, 1.0, False),
               ("r_sg2", 0.7, 0.05, 0.02, 3.0, False), ("r_f", 0.6, 0.05, 0.0, 1.0, False),
               ("c_f", 0.6, 0.05, 0.0, 1.0, False), ("b_beta", -0.05, 0.02, -5.0, 5.0, False)],
    "truth": {"c_alpha": -0.4, "r_mu1": 0.02, "r_sg1": 0.2, "r_mu2": -0.1, "r_sg2": 0.8, "r_f": 0.7,
              "c_f": 0.7, "b_beta": -0.1},
    "model": {"op": "add", "par": ["c_f"], "children": [
        {"op": "conv", "obs": "x", "grid": 400, "d_lo": -3.0, "d_hi": 3.0, "children": [
            {"op": "exp", "obs": "x", "par": ["c_alpha"]},
            {"op": "add", "par": ["r_f"], "children": [
                {"op": "gauss", "obs": "x", "par": ["r_mu1", "r_sg1"]},
                {"op": "gauss", "obs": "x", "par": ["r_mu2", "r_sg2"]}]}]},
        {"op": "exp", "obs": "x", "par": ["b_beta"]}]},
    "n_events": 1_000_000,
    "seed": 34,
}

# ---------------------------------------------------------------- COMP
# Function composition (CompositePdf): a Gaussian shell of a quadratic core,
# P(x) ~ exp(-(g(x) - mu)^2 / (2 sigma^2)), g(x) = 1 + a1 (x - 5) + a2 (x - 5)^2.
COMP = {
    "name": "comp_gauss_of_quadratic",
    "obs": [("x", 0.0, 10.0)],
    "params": [("g_a1", 0.4, 0.02, 0.0, 0.0, False), ("g_a2", 0.04, 0.005, 0.0, 0.0, False),
               ("s_mu", 2.2, 0.05, -5.0, 10.0, False), ("s_sigma", 1.0, 0.05, 0.05, 5.0, False)],
    "truth": {"g_a1": 0.5, "g_a2": 0.05, "s_mu": 2.0, "s_sigma": 1.0},
    "model": {"op": "comp", "obs": "x", "children": [
        {"op": "poly", "obs": "x", "par": ["g_a1", "g_a2"], "x0": 5.0},
        {"op": "gauss", "obs": "x", "par": ["s_mu", "s_sigma"]}]},
    "n_events": 1_000_000,
    "seed": 28,
}

# ---------------------------------------------------------------- C5
# Stream of toy fits of the C1 model with uneven event counts.
C5 = {
    "name": "c5_serving",
    "base": C1,
    "n_requests": 4096,
    "n_range": (1_000, 1_000_000),
    "rate_hz": 200.0,
    "jitter": 0.10,
    "seed": 5,
}

# ---------------------------------------------------------------- Listing 2
# Product of two exponentials in x and y (the paper's second listing).
LISTING2 = {
    "name": "listing2_prod",
    "obs": [("x", 0.0, 10.0), ("y", 0.0, 10.0)],
    "params": [("alpha_x", -2.4, 0.1, -10.0, 10.0, False),
               ("alpha_y", -1.1, 0.1, -10.0, 10.0, False)],
    "truth": {"alpha_x": -0.5, "alpha_y": -1.0},
    "model": {"op": "prod", "children": [
        {"op": "exp", "obs": "x", "par": ["alpha_x"]},
        {"op": "exp", "obs": "y", "par": ["alpha_y"]},
    ]},
    "n_events": 100_000,
    "seed": 11,
}


def workload(name):
    return {"c1": C1, "c2": C2, "c3": C3, "c4": C4, "c4x": C4X, "listing2": LISTING2, "mapped": MAPPED,
            "mapped_sum": MAPPED_SUM, "shared": SHARED, "shared_sum": SHARED_SUM, "shared_2d": SHARED_2D,
            "c4s": C4S, "c4f": C4F, "conv": CONV, "conv_poly": CONV_POLY, "comp": COMP, "conv_gmix": CONV_GMIX}[name]
