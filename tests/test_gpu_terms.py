"""Per-event parity: ln P_i and d ln P_i / d theta from the evaluation
kernels (nll_terms: the likelihood kernels run with one event per thread,
writing each event's terms instead of summing them) against the oracle's
per-event values, event by event, for every workload in both precisions.

The oracle is given the events as the dataset stores them (FP32-eval: the
float offset from the column reference, plus the reference), so range,
cell and residual-window decisions are taken on the same values on both
sides; the edge-case tests put events on, and one ulp either side of, MAP
range boundaries, DPMAP cell boundaries and CONV residual-window edges.

Per-event bounds:
  |d ln P_i|     <= TOL_L[prec] * (1 + |ln P_i|) * k_i
  |d (dlnP_ij)|  <= TOL_G[prec] * (|dlnP_ij| + mean_i |dlnP_ij|) * k_i
with k_i = 1, except for the amplitude workloads, where k_i is the
condition number of the event's amplitude sum, (1 + sum_k |c_k A_k|) / |A|
(and, time-dependent, the larger of those of A and Abar), from the oracle.
The bounds come from the arithmetic: a chain of about 32 roundings of
relative size u per event value (u = 2^-53 in double, 2^-24 in float, the
float path also seeing most parameters rounded to float) gives 32 u ~ 4e-15
(FP64) and ~2e-6 (FP32); the FP64 time-dependent terms with x add the
series approximation of the complex error function (~1e-15 relative), and
the FP32 gradients of the numerical convolution sum up to a few hundred
float terms.  So TOL_L = 5e-14 / 4e-6 and TOL_G = 5e-13 / 5e-5; the largest
values seen over every workload were 6.2e-15 / 6.8e-7 (ln P) and 5.0e-14 /
1.2e-5 (gradient).
"""
import copy

import numpy as np
import pytest

import synthgen as S
from helpers import full_data, gen_data, get_spec, oracle_for, perturbed_theta, stored_order, stored_values

pytestmark = pytest.mark.gpu

TOL_L = {"fp64": 5e-14, "fp32": 4e-6}
TOL_G = {"fp64": 5e-13, "fp32": 5e-5}

NAMES = ["c1", "c2", "listing2", "poly", "c3", "c4", "c4x", "mapped", "mapped_sum", "shared", "shared_sum",
         "shared_2d", "c4s", "conv", "conv_poly", "comp", "conv_gmix"]
AMP = {"c3", "c4", "c4x", "c4s"}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1311_1753_amd as P
    return P


def amp_condition(om, th, sdata, name):
    """(1 + sum_k |c_k A_k|) / |A| per event, from the oracle's amplitudes
    (time-dependent: the larger of A's and Abar's)."""
    if name not in AMP:
        return np.ones(len(next(iter(sdata.values()))))
    s12, s13 = sdata["s12"], sdata["s13"]
    ks = []
    for sw in (False, True) if name != "c3" else (False,):
        a, b = (s13, s12) if sw else (s12, s13)
        amp2 = om.dalitz_amp2(th, a, b)
        mag = om.dalitz_abs_terms(th, a, b)
        ks.append(mag / np.sqrt(np.maximum(amp2, 1e-300)))
    return np.maximum.reduce(ks)


def compare_terms(P, name, sp, om, g, data, prec, th, stats=None):
    ds = P.Dataset(g, data, prec)
    lp, rows = P.nll_terms(g, ds, th)
    order = stored_order(sp, data)
    sdata = {k: v[order] for k, v in stored_values(sp, data, prec).items()}
    lp_ref, rows_ref = om.logpdf(th, sdata, grad_rows=True)
    free = g.free_mask()
    # events where the density is zero (ln P = -inf) must be the same ones
    fin = np.isfinite(lp_ref)
    assert np.array_equal(np.isfinite(lp), fin), (name, prec, int((np.isfinite(lp) != fin).sum()))
    lp, lp_ref, rows, rows_ref = lp[fin], lp_ref[fin], rows[fin], rows_ref[fin]
    kappa = amp_condition(om, th, {k: v[fin] for k, v in sdata.items()}, name)
    el = np.abs(lp - lp_ref) / ((1.0 + np.abs(lp_ref)) * kappa)
    rows_ref = rows_ref[:, free]
    sc = np.abs(rows_ref) + np.abs(rows_ref).mean(axis=0)
    eg = np.abs(rows[:, free] - rows_ref) / (np.maximum(sc, 1e-300) * kappa[:, None])
    eg_max = eg.max(axis=1) if eg.size else np.zeros(lp.size)
    # the summed evaluation is the sum of these terms
    if fin.all():
        v, gr = P.nll_grad(g, ds, th)
        tol_sum = 1e-13 if prec == "fp64" else 1e-6
        assert abs(v + lp.sum()) <= tol_sum * max(1.0, np.abs(lp).sum()), (v, -lp.sum())
        gl1 = np.abs(rows[:, free]).sum(axis=0) + 1e-300
        assert np.all(np.abs(gr[free] + rows[:, free].sum(axis=0)) <= tol_sum * gl1)
    ds.free()
    if lp.size:
        i = int(np.argmax(np.maximum(el, eg_max)))
        print(f"  {name} {prec} n={len(lp)}: lnP err max {el.max():.2e} p99.9 {np.quantile(el, 0.999):.2e}; "
              f"grad err max {eg_max.max():.2e} p99.9 {np.quantile(eg_max, 0.999):.2e}; worst event {i} "
              f"lnP {lp[i]:.6g} ref {lp_ref[i]:.6g} kappa {kappa[i]:.3g}", flush=True)
    if stats is not None:
        stats.append((name, prec, float(el.max(initial=0)), float(eg_max.max(initial=0))))
    assert np.all(el <= TOL_L[prec]), (name, prec, float(el.max()), int(np.argmax(el)))
    assert np.all(eg_max <= TOL_G[prec]), (name, prec, float(eg_max.max()), int(np.argmax(eg_max)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", NAMES)
def test_terms_match_oracle_event_by_event(P, name, prec):
    print(f"\n[case] terms {name} {prec}", flush=True)
    sp = get_spec(name)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    n = 20_011 if name not in AMP else 8_009
    data = gen_data(name, n, 500 + NAMES.index(name))
    for k, th in enumerate([om.theta(sp["truth"]), perturbed_theta(om, sp, seed=77)]):
        compare_terms(P, name, sp, om, g, data, prec, th)


def _nb(x):
    """x and its two neighbouring doubles."""
    return [np.nextafter(x, -np.inf), x, np.nextafter(x, np.inf)]


def _map_edges():
    out = []
    for b in S.MAPPED["model"]["bounds"]:
        out += _nb(b)
        # values whose FP32-eval offset (from the box middle, 5) rounds onto the boundary
        out += [b + 1e-8, b - 1e-8, b + 2.9e-8, b - 2.9e-8]
    return np.array(out)


def _conv_edges(spc):
    lo, hi, N = 0.0, 10.0, spc["grid"]
    h = (hi - lo) / N
    out = []
    for k in (0, 1, 7, N // 3, N // 2, N - 2, N - 1):
        t = lo + (k + 0.5) * h
        for d in (spc["d_lo"], spc["d_hi"]):
            x = t + d
            if lo <= x <= hi:
                out += _nb(x) + [x + 1e-9, x - 1e-9]
    return np.clip(np.array(out), lo, hi)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["mapped", "mapped_sum", "conv", "conv_poly", "conv_gmix", "c4s"])
def test_terms_on_range_and_window_edges(P, name, prec):
    """Events on and next to the boundaries where a range, a cell or a
    residual-window decision changes, mixed into ordinary events."""
    print(f"\n[case] terms edges {name} {prec}", flush=True)
    sp = get_spec(name)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    base = gen_data(name, 2_003, 900 + len(name))
    if name in ("mapped", "mapped_sum"):
        x = np.concatenate([base["x"], _map_edges()])
        data = {"x": x}
    elif name in ("conv", "conv_poly", "conv_gmix"):
        spc = sp["model"] if sp["model"]["op"] == "conv" else sp["model"]["children"][0]
        data = {"x": np.concatenate([base["x"], _conv_edges(spc)])}
    else:
        # s12 / s13 on the cell boundary (and one ulp either side), inside the plot
        b12, b13 = S.SIGMA_T_BOUNDS[0][0], S.SIGMA_T_BOUNDS[1][0]
        s12, s13 = [], []
        for a in _nb(b12):
            for c in (0.9, 1.2, 1.4, 1.6, 2.0):
                s12.append(a)
                s13.append(c)
        for c in _nb(b13):
            for a in (0.9, 1.2, 1.4, 1.6, 2.0):
                s12.append(a)
                s13.append(c)
        s12, s13 = np.array(s12), np.array(s13)
        # the oracle's membership rule: |A|^2 = 1 inside with every coefficient 0
        inside = om.dalitz_amp2(np.zeros(g.n_par), s12, s13) > 0
        s12, s13 = s12[inside], s13[inside]
        m = s12.size
        rng = np.random.default_rng(5)
        st = rng.uniform(0.02, 0.2, m)
        t = rng.exponential(0.41, m) + st * rng.standard_normal(m)
        data = {"s12": np.concatenate([base["s12"], s12]), "s13": np.concatenate([base["s13"], s13]),
                "t": np.concatenate([base["t"], t]), "sigma_t": np.concatenate([base["sigma_t"], st])}
    for th in (om.theta(sp["truth"]), perturbed_theta(om, sp, seed=78)):
        compare_terms(P, name, sp, om, g, data, prec, th)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 300_001])
def test_terms_row_tails(P, n, prec):
    """Empty and one-event datasets, partial and exact chunks, and more than
    one terms launch (2^18 events each)."""
    print(f"\n[case] terms tails c2 n={n} {prec}", flush=True)
    sp = get_spec("c2")
    om = oracle_for("c2")
    g = P.Graph.from_spec(sp)
    data = gen_data("c2", n, 60 + n % 89) if n else {"x": np.zeros(0)}
    th = perturbed_theta(om, sp, seed=61)
    if n == 0:
        ds = P.Dataset(g, data, prec)
        lp, rows = P.nll_terms(g, ds, th)
        assert lp.shape == (0,) and rows.shape == (0, g.n_par)
        ds.free()
        return
    compare_terms(P, "c2", sp, om, g, data, prec, th)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c4x", "c4s"])
def test_terms_sampled_at_full_size(P, name):
    """The workloads at full size (10^7 composite events, 10^6 Dalitz
    events, 2x10^6 time-dependent events): terms of every event from the
    kernels, 20000 sampled events compared with the oracle one by one, and
    the terms' sum against nll_grad over the whole dataset."""
    print(f"\n[case] terms full-size {name} sampled", flush=True)
    sp = get_spec(name)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    data = full_data(name)
    n = len(next(iter(data.values())))
    th = perturbed_theta(om, sp, rel=0.01, seed=3)
    idx = np.sort(np.random.default_rng(8).choice(n, 20_000, replace=False))
    free = g.free_mask()
    for prec in ("fp32", "fp64"):
        ds = P.Dataset(g, data, prec)
        lp, rows = P.nll_terms(g, ds, th)
        v, _ = P.nll_grad(g, ds, th)
        ds.free()
        sd = {k: v_[idx] for k, v_ in stored_values(sp, data, prec).items()}
        lp_ref, rows_ref = om.logpdf(th, sd, grad_rows=True)
        kappa = amp_condition(om, th, sd, name)
        el = np.abs(lp[idx] - lp_ref) / ((1.0 + np.abs(lp_ref)) * kappa)
        rr = rows_ref[:, free]
        sc = np.abs(rr) + np.abs(rr).mean(axis=0)
        eg = np.abs(rows[idx][:, free] - rr) / (np.maximum(sc, 1e-300) * kappa[:, None])
        print(f"  {prec}: lnP err max {el.max():.2e}; grad err max {eg.max():.2e} (component "
              f"{int(np.argmax(eg.max(axis=0)))})", flush=True)
        assert el.max() <= TOL_L[prec] and eg.max() <= TOL_G[prec]
        assert abs(v + lp.sum()) <= (1e-13 if prec == "fp64" else 1e-6) * np.abs(lp).sum()


def _conv_variant(grid, second):
    """The CONV workload with another grid size, or (second) with its
    background replaced by a second convolution (the background exponential
    smeared by the same Gaussian on a 300-point grid)."""
    sp = copy.deepcopy(S.configs.CONV)
    sp["name"] = f"conv_grid{grid}" + ("_two" if second else "")
    sp["model"]["children"][0]["grid"] = grid
    if second:
        sp["model"]["children"][1] = {"op": "conv", "obs": "x", "grid": 300, "d_lo": -2.0, "d_hi": 2.0, "children": [
            {"op": "exp", "obs": "x", "par": ["b_beta"]},
            {"op": "gauss", "obs": "x", "par": ["r_mu", "r_sigma"]}]}
    return sp


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("grid,second", [(512, False), (513, False), (400, True)])
def test_terms_conv_staged_and_direct_model(P, grid, second, prec):
    """A row stages the model of a graph's one CONV node in LDS when its grid
    has at most 512 points; a larger grid, or a second CONV node, takes the
    interpreter that evaluates the model per term.  Both at the limit and
    either side of it, per event against the oracle (edge events included)."""
    from oracle import oracle as O
    print(f"\n[case] terms conv grid={grid} second={second} {prec}", flush=True)
    sp = _conv_variant(grid, second)
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    rng = np.random.default_rng(grid + 7 * second)
    x = np.concatenate([rng.uniform(0.0, 10.0, 6_007), _conv_edges(sp["model"]["children"][0])])
    data = {"x": x}
    for th in (om.theta(sp["truth"]), perturbed_theta(om, sp, seed=79)):
        compare_terms(P, sp["name"], sp, om, g, data, prec, th)


def _conv_gmix_times_exp_y():
    """The two-Gaussian-resolution convolution workload times an exponential
    in a second observable: 9 slots, more than the small staged-CONV kernel
    takes, so the general staged-CONV interpreter evaluates it."""
    base = S.configs.CONV_GMIX
    return {
        "name": "conv_gmix_times_exp_y",
        "obs": list(base["obs"]) + [("y", 0.0, 5.0)],
        "params": list(base["params"]) + [("y_alpha", -0.4, 0.05, -5.0, 5.0, False)],
        "truth": dict(base["truth"], y_alpha=-0.5),
        "model": {"op": "prod", "children": [copy.deepcopy(base["model"]),
                                             {"op": "exp", "obs": "y", "par": ["y_alpha"]}]},
    }


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_terms_conv_staged_general_interpreter(P, prec):
    """A CONV graph beyond the small kernel's 8 slots (the general staged-CONV
    interpreter), per event against the oracle, window-edge events included."""
    from oracle import oracle as O
    print(f"\n[case] terms conv_gmix x exp(y) {prec}", flush=True)
    sp = _conv_gmix_times_exp_y()
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    assert g.n_par == 9
    rng = np.random.default_rng(97)
    x = np.concatenate([rng.uniform(0.0, 10.0, 6_011), _conv_edges(sp["model"]["children"][0]["children"][0])])
    data = {"x": x, "y": rng.uniform(0.0, 5.0, x.size)}
    for th in (om.theta(sp["truth"]), perturbed_theta(om, sp, seed=81)):
        compare_terms(P, sp["name"], sp, om, g, data, prec, th)


def _conv_three_gauss_resolution():
    """An exponential smeared by a resolution of three Gaussians (core, wider
    and tail), each normalised over the residual range: 9 slots, the general
    staged-CONV interpreter's loop for three components."""
    return {
        "name": "conv_exp_three_gauss",
        "obs": [("x", 0.0, 10.0)],
        "params": [("c_alpha", -0.3, 0.05, -5.0, 5.0, False),
                   ("r_mu1", 0.0, 0.02, -1.0, 1.0, False), ("r_sg1", 0.2, 0.02, 0.02, 2.0, False),
                   ("r_mu2", 0.0, 0.02, -1.0, 1.0, False), ("r_sg2", 0.5, 0.05, 0.02, 3.0, False),
                   ("r_mu3", 0.0, 0.02, -1.0, 1.0, False), ("r_sg3", 1.0, 0.05, 0.02, 3.0, False),
                   ("r_f1", 0.6, 0.05, 0.0, 1.0, False), ("r_f2", 0.3, 0.05, 0.0, 1.0, False)],
        "truth": {"c_alpha": -0.4, "r_mu1": 0.02, "r_sg1": 0.2, "r_mu2": -0.05, "r_sg2": 0.5,
                  "r_mu3": 0.1, "r_sg3": 1.1, "r_f1": 0.6, "r_f2": 0.3},
        "model": {"op": "conv", "obs": "x", "grid": 400, "d_lo": -3.0, "d_hi": 3.0, "children": [
            {"op": "exp", "obs": "x", "par": ["c_alpha"]},
            {"op": "add", "par": ["r_f1", "r_f2"], "children": [
                {"op": "gauss", "obs": "x", "par": ["r_mu1", "r_sg1"]},
                {"op": "gauss", "obs": "x", "par": ["r_mu2", "r_sg2"]},
                {"op": "gauss", "obs": "x", "par": ["r_mu3", "r_sg3"]}]}]},
    }


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_terms_conv_three_gaussian_resolution(P, prec):
    """A three-Gaussian resolution mixture, per event against the oracle,
    window-edge events included."""
    from oracle import oracle as O
    print(f"\n[case] terms conv three-Gaussian resolution {prec}", flush=True)
    sp = _conv_three_gauss_resolution()
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    rng = np.random.default_rng(113)
    x = np.concatenate([rng.uniform(0.0, 10.0, 6_007), _conv_edges(sp["model"])])
    data = {"x": x}
    for th in (om.theta(sp["truth"]), perturbed_theta(om, sp, seed=83)):
        compare_terms(P, sp["name"], sp, om, g, data, prec, th)
