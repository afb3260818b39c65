"""The full time-dependent model of the mixing fit (section "Results": 16
complex amplitudes, x and y, complex q/p, floating resonance masses and
widths) on the GPU against the oracle: per-event ln P and d ln P / d theta
(nll_terms) event by event, and the summed NLL and gradient, in both
precisions, with floating shapes (normalisation re-computed by the grid
kernel at every evaluation) and with fixed shapes (grid matrices for 16
amplitudes, q/p applied to them).

Per-event bounds as for the other amplitude workloads (see test_gpu_terms:
|d ln P_i| <= TOL_L (1 + |ln P_i|) k_i, the gradient relative to
|dlnP_ij| + mean_i |dlnP_ij|, k_i the condition number of the event's
amplitude sums); summed results within 1e-12 (FP64) and 1e-6 (FP32) of
the sum of |ln P_i| and of each gradient component's scale: the sum over
events of its per-event scale (below) times k_i, plus n |d ln N / d theta_j|
(the per-event bounds summed; each event's derivative is its own term minus
the normalisation's, and the summed gradient carries the normalisation's
rounding n times, whatever the events' terms cancel).

The |q/p| and arg q/p derivatives, (|Abar'|^2 (C - Cz) + a_s S + b_s Sz) /
(|q/p| R) and (a_s Sz - b_s S) / R, hold the difference C - Cz of two decay
-time factors that nearly coincide at small t (they differ by terms of order
y t / tau); each side forms them with different algorithms (the closed form
with erfcx, and the complex error function or the oscillating integral),
each good to about 3e-15 relative, so the absolute error of these columns
scales with |Abar'|^2 E(t) / R (E the convolved decay) and not with their
value.  Their per-event scale, and the scale of their sums, add that
magnitude."""
import copy

import numpy as np
import pytest

import synthgen as S
from helpers import stored_values

pytestmark = pytest.mark.gpu

TOL_L = {"fp64": 5e-14, "fp32": 4e-6}
TOL_G = {"fp64": 5e-13, "fp32": 5e-5}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1311_1753_amd as P
    return P


def full_spec(floating=True, grid=100):
    sp = S.configs._full_model(grid=grid)
    if not floating:
        node = sp["model"]
        for r in node["dalitz"]["resonances"]:
            r.pop("float", None)
        keep = node["par"][:35]
        node["par"] = keep
        sp["params"] = [p for p in sp["params"] if p[0] in keep]
        sp["truth"] = {k: v for k, v in sp["truth"].items() if k in keep}
    return sp


def points(sp, n, seed):
    """Events uniform over the Dalitz plot, decay times exponential plus
    resolution, sigma_t ~ U[0.02, 0.2] (the shapes of the time-dependent
    workloads' full-size samples)."""
    from oracle import oracle as O
    om = O.Model(full_spec(True, grid=10))  # membership only: |A|^2 = 1 inside at c = 0
    zero = np.zeros(len(om.par_names))
    lo, hi = S.dalitz_box()
    rng = np.random.default_rng(seed)
    a, b = [], []
    got = 0
    while got < n:
        u = rng.uniform(lo, hi, 4 * n + 64)
        v = rng.uniform(lo, hi, 4 * n + 64)
        keep = om.dalitz_amp2(zero, u, v) > 0
        a.append(u[keep])
        b.append(v[keep])
        got += int(keep.sum())
    st = rng.uniform(0.02, 0.2, n)
    t = rng.exponential(0.41, n) + st * rng.standard_normal(n)
    return {"s12": np.concatenate(a)[:n], "s13": np.concatenate(b)[:n], "t": t, "sigma_t": st}


def theta_off(om, sp, seed=3):
    rng = np.random.default_rng(seed)
    th = om.theta(sp["truth"])
    th[:30] *= 1.0 + 0.2 * rng.standard_normal(30)
    i = om.par_names.index
    th[i("tau")], th[i("y")], th[i("x")] = 0.43, 0.06, 0.05
    th[i("qp_mag")], th[i("qp_phase")] = 0.85, 0.4
    if "rho_m0" in om.par_names:
        th[i("rho_m0")], th[i("rho_g0")] = 0.781, 0.143
        th[i("kst_m0")], th[i("kst_g0")] = 0.889, 0.054
    return th


def qp_scale(om, th, d):
    """|q/p|^2 |Abar|^2 E(t; 1/tau, sigma_t) / R per event, from the oracle
    (amplitudes at the fixed shapes: a magnitude for the bound only)."""
    i = om.par_names.index
    ab2 = om.dalitz_amp2(th, d["s13"], d["s12"])
    tau = th[i("tau")]
    E = np.fromiter((om_econv(t, 1.0 / tau, s) for t, s in zip(d["t"], d["sigma_t"])), float, len(d["t"]))
    lnN = om.node_lnnorm(om.root, th)[0]
    R = np.exp(om.logpdf(th, d) + lnN)
    return th[i("qp_mag")] ** 2 * ab2 * E / R


def om_econv(t, G, s):
    from oracle import oracle as O
    return O.econv(t, G, s)


def condition(om, th, d):
    s12, s13 = d["s12"], d["s13"]
    ks = []
    for a, b in ((s12, s13), (s13, s12)):
        amp2 = om.dalitz_amp2(th, a, b)
        ks.append(om.dalitz_abs_terms(th, a, b) / np.sqrt(np.maximum(amp2, 1e-300)))
    return np.maximum.reduce(ks)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("floating", [True, False])
def test_full_model_terms_and_sums(P, floating, prec):
    from oracle import oracle as O
    print(f"\n[case] full tddp floating={floating} {prec}", flush=True)
    sp = full_spec(floating)
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    data = points(sp, 6007, 11 + floating)
    free = g.free_mask()
    for th in (om.theta(sp["truth"]), theta_off(om, sp)):
        ds = P.Dataset(g, data, prec)
        lp, rows = P.nll_terms(g, ds, th)
        sd = stored_values(sp, data, prec)
        lp_ref, rows_ref = om.logpdf(th, sd, grad_rows=True)
        assert np.all(np.isfinite(lp)) and np.all(np.isfinite(lp_ref))
        kappa = condition(om, th, sd)
        el = np.abs(lp - lp_ref) / ((1.0 + np.abs(lp_ref)) * kappa)
        sc_all = np.abs(rows_ref) + np.abs(rows_ref).mean(axis=0)
        q = qp_scale(om, th, sd)
        for name in ("qp_mag", "qp_phase"):
            sc_all[:, om.par_names.index(name)] += q
        rr = rows_ref[:, free]
        sc = sc_all[:, free]
        eg = (np.abs(rows[:, free] - rr) / (np.maximum(sc, 1e-300) * kappa[:, None])).max(axis=1)
        print(f"  lnP err max {el.max():.2e}; grad err max {eg.max():.2e}", flush=True)
        assert np.all(el <= TOL_L[prec]), (float(el.max()), int(np.argmax(el)))
        assert np.all(eg <= TOL_G[prec]), (float(eg.max()), int(np.argmax(eg)))
        # the summed evaluation against the oracle's NLL and gradient
        v, gr = P.nll_grad(g, ds, th)
        vr, grr = om.nll(th, sd, grad=True)
        tol = 1e-12 if prec == "fp64" else 1e-6
        assert abs(v - vr) <= tol * np.abs(lp_ref).sum(), (v, vr)
        gl1 = (kappa[:, None] * sc_all).sum(axis=0) + 1e-300 + len(lp_ref) * np.abs(om.node_lnnorm(om.root, th)[1])
        err = np.abs(gr - grr)[free] / gl1[free]
        print(f"  sums: NLL err {abs(v - vr) / np.abs(lp_ref).sum():.2e}, grad err max {err.max():.2e}", flush=True)
        assert np.all(err <= tol), (float(err.max()), om.par_names[int(np.argmax(err))])
        ds.free()


def test_full_model_repeatable_and_domain(P):
    """Two evaluations give the same bits (the grid sums and the event sums
    have fixed orders); |q/p| <= 0 or a mass below threshold is a domain
    error, not a NaN."""
    from oracle import oracle as O
    print("\n[case] full tddp repeat/domain", flush=True)
    sp = full_spec(True)
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, points(sp, 3001, 5), "fp32")
    th = theta_off(om, sp)
    v1, g1 = P.nll_grad(g, ds, th)
    v2, g2 = P.nll_grad(g, ds, th)
    assert v1 == v2 and np.array_equal(g1, g2)
    for name, val in (("qp_mag", 0.0), ("rho_m0", 0.2)):
        bad = th.copy()
        bad[om.par_names.index(name)] = val
        with pytest.raises(P.HipfitError):
            P.nll_grad(g, ds, bad, allow_domain=False)
        v, gr = P.nll_grad(g, ds, bad)
        assert v == np.inf
    ds.free()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_model_fit_matches_oracle_fit(P, prec):
    """The 39-parameter fit on the GPU (the project's minimiser, analytic
    gradient) against the oracle's fit of the same 5 x 10^4 events from the
    same start (tests/golden/tddp_full_fit.json, written by
    make_tddp_full_fit.py from the oracle alone): parameters within 1e-3
    sigma, errors within 2e-3 relative."""
    import json
    import os
    from helpers import gen_data, get_spec, oracle_for
    print(f"\n[case] full tddp fit {prec}", flush=True)
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "tddp_full_fit.json")))["fit"]
    sp = get_spec(ref["name"])
    om = oracle_for(ref["name"])
    assert np.allclose(om.theta(), ref["start"], rtol=0, atol=0)
    assert [p[0] for p in sp["params"]] == ref["par_names"]
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, gen_data(ref["name"], ref["n_events"], ref["seed"]), prec)
    r = P.fit(g, ds)
    free = g.free_mask()
    th_ref, err_ref = np.array(ref["theta"]), np.array(ref["errors"])
    dev = np.abs(r["theta"] - th_ref)[free] / err_ref[free]
    rel_err = np.abs(r["errors"][free] / err_ref[free] - 1.0)
    print(f"  status {r['status']} n_eval {r['n_eval']} nll {r['nll']:.10f} (oracle {ref['nll']:.10f}) "
          f"max |dtheta|/sigma {dev.max():.2e} ({sp['params'][int(np.argmax(dev))][0]}) "
          f"max error ratio - 1 {rel_err.max():.2e}", flush=True)
    assert r["status"] == "OK"
    assert dev.max() <= 1e-3, "different minimum" if dev.max() > 1.0 else dev.max()
    assert rel_err.max() <= 2e-3
    ds.free()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_model_full_size(P, prec):
    """The benchmark's full model (normalisation grid 1000 x 1000, 10^6
    events uniform over the plot with exponential decay times, as the
    benchmark times it) at a parameter point off the truth: summed NLL and
    gradient against the oracle's, with the bounds of the small-size test."""
    from oracle import oracle as O
    print(f"\n[case] full tddp full size {prec}", flush=True)
    sp = S.configs._full_model()
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    data = points(sp, sp["n_events"], sp["seed"])
    th = theta_off(om, sp)
    ds = P.Dataset(g, data, prec)
    v, gr = P.nll_grad(g, ds, th)
    sd = stored_values(sp, data, prec)
    lp_ref, rows_ref = om.logpdf(th, sd, grad_rows=True)
    vr, grr = -lp_ref.sum(), -rows_ref.sum(axis=0)
    q = qp_scale(om, th, sd)
    kappa = condition(om, th, sd)
    sc_all = np.abs(rows_ref) + np.abs(rows_ref).mean(axis=0)
    for name in ("qp_mag", "qp_phase"):
        sc_all[:, om.par_names.index(name)] += q
    gl1 = (kappa[:, None] * sc_all).sum(axis=0) + 1e-300 + len(lp_ref) * np.abs(om.node_lnnorm(om.root, th)[1])
    free = g.free_mask()
    tol = 1e-12 if prec == "fp64" else 1e-6
    err = np.abs(gr - grr)[free] / gl1[free]
    print(f"  n={ds.n} NLL err {abs(v - vr) / np.abs(lp_ref).sum():.2e}, grad err max {err.max():.2e} "
          f"({om.par_names[int(np.argmax(np.abs(gr - grr) / gl1))]})", flush=True)
    assert abs(v - vr) <= tol * np.abs(lp_ref).sum()
    assert np.all(err <= tol)
    ds.free()


@pytest.mark.parametrize("floating", [True, False])
def test_full_model_nll_only_empty_and_noalloc(P, floating):
    """The NLL-only evaluation (the grid kernel without derivatives) against
    the oracle in both precisions; an empty dataset gives NLL 0 and a zero
    gradient; the allocation-free entry point gives nll_grad's bits with
    fixed shapes and refuses floating ones (their grid kernel needs its own
    partial rows)."""
    import torch
    from oracle import oracle as O
    print(f"\n[case] full tddp nll-only/empty/noalloc floating={floating}", flush=True)
    sp = full_spec(floating)
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    data = points(sp, 4001, 21)
    th = theta_off(om, sp)
    for prec in ("fp64", "fp32"):
        ds = P.Dataset(g, data, prec)
        v = P.nll_eval(g, ds, th)
        sd = stored_values(sp, data, prec)
        lp_ref = om.logpdf(th, sd)
        tol = 1e-12 if prec == "fp64" else 1e-6
        assert abs(v + lp_ref.sum()) <= tol * np.abs(lp_ref).sum(), (prec, v, -lp_ref.sum())
        v2, gr2 = P.nll_grad(g, ds, th)
        assert abs(v2 - v) <= tol * np.abs(lp_ref).sum()
        cols = {}
        for name, x in data.items():
            x = np.asarray(x, dtype=np.float64)
            if prec == "fp64":
                cols[name] = torch.tensor(x, dtype=torch.float64, device="cuda")
            else:
                ref = g.column_ref(name, "fp32")
                cols[name] = torch.tensor((x - ref).astype(np.float32), dtype=torch.float32, device="cuda")
        if floating:
            with pytest.raises(P.HipfitError):
                P.nll_grad_noalloc(g, cols, th, precision=prec)
        else:
            v3, gr3 = P.nll_grad_noalloc(g, cols, th, precision=prec)
            assert v3 == v2 and np.array_equal(gr3, gr2)
        ds.free()
    empty = P.Dataset(g, {k: v[:0] for k, v in data.items()}, "fp64")
    v, gr = P.nll_grad(g, empty, th)
    assert v == 0.0 and not np.any(gr)
    empty.free()
