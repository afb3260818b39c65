"""Shared test helpers: workload data at test sizes and tolerance scales.

Data come from the seeded generators in synthgen; where a density is needed
for accept-reject (the Dalitz workloads) it is the oracle's, so no test input
ever comes from the GPU path."""
import copy
import functools
import math

import numpy as np

import synthgen as S


def full_fit_spec():
    """The full time-dependent model (15 resonances and the non-resonant
    term, x, y, complex q/p, two floating shapes) at a test size: a 200 x 200
    normalisation grid, mixing parameters y = 0.1, x = 0.08 so that q/p is
    constrained by 5 x 10^4 events, starts at y = 0.09, x = 0.07."""
    sp = S.configs._full_model(grid=200, n_events=50_000, seed=9)
    sp["name"] = "c4f_fit"
    sp["truth"] = dict(sp["truth"], y=0.1, x=0.08)
    start = {"y": 0.09, "x": 0.07}
    sp["params"] = [(p[0], start.get(p[0], p[1])) + tuple(p[2:]) for p in sp["params"]]
    return sp


def spec(name):
    if name == "c4f_fit":
        return full_fit_spec()
    return copy.deepcopy(S.workload(name))


@functools.lru_cache(maxsize=None)
def _oracle_model(name):
    from oracle import oracle as O
    return O.Model(spec(name))


def oracle_model(name):
    return _oracle_model(name)


def gen_data(name, n, seed):
    """Events of workload `name` (dict of float64 columns)."""
    if name == "c1":
        return S.gen_c1(n=n, seed=seed)
    if name == "c2":
        return S.gen_c2(n=n, seed=seed)
    if name == "listing2":
        return S.gen_listing2(n=n, seed=seed)
    if name == "poly":
        rng = np.random.default_rng(seed)
        return {"x": rng.uniform(-1.0, 3.0, n)}
    if name == "c4s":
        # the C4 events with sigma_t drawn from the density of the event's cell
        m = oracle_model("c4")
        th = m.theta(S.workload("c4")["truth"])
        lo, hi = S.dalitz_box()
        G = 200
        c = lo + (np.arange(G) + 0.5) * (hi - lo) / G
        a, b = np.meshgrid(c, c, indexing="ij")
        env = 1.3 * (m.dalitz_amp2(th, a.ravel(), b.ravel()) + m.dalitz_amp2(th, a.ravel(), b.ravel(),
                                                                               swapped=True)).max()
        cells = (S.SIGMA_T_BOUNDS[0], S.SIGMA_T_BOUNDS[1], S.SIGMA_T_CELLS)
        return S.gen_accept_reject_tddp(n, seed, lambda x, yy, t: m.tddp_rate(th, x, yy, t), env, th[-2], th[-1],
                                        batch=1 << 18, sigma_t_cells=cells)
    if name in ("c3", "c4", "c4x", "c4f_fit"):
        m = oracle_model(name)
        th = m.theta(spec(name)["truth"])
        lo, hi = S.dalitz_box()
        G = 200
        c = lo + (np.arange(G) + 0.5) * (hi - lo) / G
        a, b = np.meshgrid(c, c, indexing="ij")
        if name == "c3":
            env = 1.3 * m.dalitz_amp2(th, a.ravel(), b.ravel()).max()
            return S.gen_accept_reject_dalitz(n, seed, lambda x, y: m.dalitz_amp2(th, x, y), env,
                                              batch=1 << 18)
        a2 = m.dalitz_amp2(th, a.ravel(), b.ravel())
        b2 = m.dalitz_amp2(th, a.ravel(), b.ravel(), swapped=True)
        # the rate over e^{-(1-|y|) t/tau} is at most (1 + 1/sqrt2)(|A|^2 + |Abar|^2)
        env = (1.3 if name == "c4" else 1.8) * (a2 + b2).max()
        tau, y = th[m.par_names.index("tau")], th[m.par_names.index("y")]
        return S.gen_accept_reject_tddp(n, seed, lambda x, yy, t: m.tddp_rate(th, x, yy, t), env, tau, y,
                                        batch=1 << 18)
    if name in ("mapped", "mapped_sum"):
        m = oracle_model(name)
        th = m.theta(S.workload(name)["truth"])
        grid = np.linspace(0.0, 10.0, 4001)
        dens = lambda x: np.exp(m.logpdf(th, {"x": x}))
        return {"x": S.gen_accept_reject_1d(n, seed, dens, 1.2 * dens(grid).max(), 0.0, 10.0, batch=1 << 18)}
    if name == "comp":
        m = oracle_model(name)
        th = m.theta(S.workload(name)["truth"])
        grid = np.linspace(0.0, 10.0, 4001)
        dens = lambda x: np.exp(m.logpdf(th, {"x": x}))
        return {"x": S.gen_accept_reject_1d(n, seed, dens, 1.2 * dens(grid).max(), 0.0, 10.0, batch=1 << 18)}
    if name in ("conv", "conv_poly", "conv_gmix"):
        m = oracle_model(name)
        th = m.theta(S.workload(name)["truth"])
        grid = np.linspace(0.0, 10.0, 4001)
        dens = lambda x: np.exp(m.logpdf(th, {"x": x}))
        return {"x": S.gen_accept_reject_1d(n, seed, dens, 1.3 * dens(grid).max(), 0.0, 10.0, batch=1 << 18)}
    if name in ("shared", "shared_sum", "shared_2d"):
        # x from the 1-D density (the 2-D product factorises: x from the shared
        # product, y from its exponential by inverting the CDF)
        base = "shared" if name == "shared_2d" else name
        m = oracle_model(base)
        th = m.theta(S.workload(base)["truth"])
        grid = np.linspace(0.0, 10.0, 4001)
        dens = lambda x: np.exp(m.logpdf(th, {"x": x}))
        x = S.gen_accept_reject_1d(n, seed, dens, 1.2 * dens(grid).max(), 0.0, 10.0, batch=1 << 18)
        if name != "shared_2d":
            return {"x": x}
        a, L = S.SHARED_2D["truth"]["y_alpha"], 5.0
        u = np.random.default_rng(seed + 1).uniform(0.0, 1.0, n)
        return {"x": x, "y": np.log1p(u * np.expm1(a * L)) / a}
    raise ValueError(name)


_full_cache = {}


def full_data(name):
    """Events of a workload at its full size: the benchmark's 10^7-event
    composite sample, the 10^6-event Dalitz sample (accept-reject on the
    oracle's density), and for the time-dependent workloads 2x10^6 points
    uniform over the plot with exponential decay times smeared by
    sigma_t ~ U[0.02, 0.2] (shared by the x-free and sigma_t-map variants)."""
    if name in _full_cache:
        return _full_cache[name]
    if name in ("c4x", "c4s"):  # the same observables as c4
        return full_data("c4")
    if name == "c2":
        d = S.gen_c2()
    elif name == "c3":
        d = gen_data("c3", S.C3["n_events"], S.C3["seed"])
    else:
        om = oracle_for("c4")
        n = S.C4["n_events"]
        rng = np.random.default_rng(S.C4["seed"])
        lo, hi = S.dalitz_box()
        s12, s13 = [], []
        got = 0
        th = om.theta(S.C4["truth"])
        while got < n:
            a = lo + (hi - lo) * rng.random(1 << 22)
            b = lo + (hi - lo) * rng.random(1 << 22)
            keep = om.dalitz_amp2(np.zeros_like(th), a, b) > 0  # c = 0: |A|^2 = 1 inside
            s12.append(a[keep])
            s13.append(b[keep])
            got += int(keep.sum())
        s12 = np.concatenate(s12)[:n]
        s13 = np.concatenate(s13)[:n]
        st = rng.uniform(0.02, 0.2, n)
        t = rng.exponential(0.41, n) + st * rng.standard_normal(n)
        d = {"s12": s12, "s13": s13, "t": t, "sigma_t": st}
    _full_cache[name] = d
    return d


POLY_SPEC = {
    "name": "poly3",
    "obs": [("x", -1.0, 3.0)],
    "params": [("a1", 0.2, 0.05, 0.0, 0.0, False), ("a2", 0.3, 0.05, 0.0, 0.0, False),
               ("a3", -0.05, 0.01, 0.0, 0.0, False)],
    "truth": {"a1": 0.2, "a2": 0.3, "a3": -0.05},
    "model": {"op": "poly", "obs": "x", "par": ["a1", "a2", "a3"], "x0": 1.0},
}


def get_spec(name):
    if name == "poly":
        return copy.deepcopy(POLY_SPEC)
    return spec(name)


def oracle_for(name):
    from oracle import oracle as O
    if name == "poly":
        return O.Model(POLY_SPEC)
    return oracle_model(name)


def _nodes(m):
    yield m
    for c in m.get("children", []):
        yield from _nodes(c)


def column_refs(sp, prec):
    """Per observable, the reference that the FP32-eval storage subtracts
    (the documented storage format: the middle of a finite box; 0 for an
    unbounded box and for the decay time and its uncertainty of a
    time-dependent Dalitz node, which are stored as they are); 0 for FP64."""
    if prec == "fp64":
        return {o[0]: 0.0 for o in sp["obs"]}
    raw = set()
    for nd in _nodes(sp["model"]):
        if nd["op"] == "tddp":
            raw.update(nd["obs"][2:4])
    out = {}
    for name, lo, hi in sp["obs"]:
        fin = math.isfinite(lo) and math.isfinite(hi)
        out[name] = 0.5 * (lo + hi) if fin and name not in raw else 0.0
    return out


def stored_values(sp, data, prec):
    """The events as the dataset holds them: FP64 as given; FP32-eval as the
    float offset from the column reference, rounded once, plus the reference
    (what the kernels evaluate, so the oracle is given the same events)."""
    if prec == "fp64":
        return {k: np.asarray(v, dtype=np.float64) for k, v in data.items()}
    ref = column_refs(sp, prec)
    return {k: ref[k] + (np.asarray(v, dtype=np.float64) - ref[k]).astype(np.float32).astype(np.float64)
            for k, v in data.items()}


def stored_order(sp, data):
    """Event order of a dataset: graphs with a convolution node store their
    events sorted by that node's observable (stable), others as given."""
    for nd in _nodes(sp["model"]):
        if nd["op"] == "conv":
            return np.argsort(np.asarray(data[nd["obs"]]), kind="stable")
    return np.arange(len(next(iter(data.values()))))


def nll_scale(model, theta, data):
    """max(|NLL|, sum_i |ln P_i|): the scale relative tolerances refer to."""
    lp = model.logpdf(theta, data)
    return max(abs(lp.sum()), np.abs(lp).sum())


def grad_scale(model, theta, data):
    """sum_i |d ln P_i / d theta_j| (L1 scale of each gradient component)."""
    _, rows = model.logpdf(theta, data, grad_rows=True)
    return np.abs(rows).sum(axis=0)


AMP_WORKLOADS = {"c3", "c4", "c4x", "c4s"}


def amp_condition(om, th, sdata, name):
    """(1 + sum_k |c_k A_k|) / |A| per event, from the oracle's amplitudes
    (time-dependent: the larger of A's and Abar's): the factor by which the
    rounding of the terms of the amplitude sum can grow in A."""
    s12, s13 = sdata["s12"], sdata["s13"]
    ks = []
    for sw in (False, True) if name != "c3" else (False,):
        a, b = (s13, s12) if sw else (s12, s13)
        amp2 = om.dalitz_amp2(th, a, b)
        ks.append(om.dalitz_abs_terms(th, a, b) / np.sqrt(np.maximum(amp2, 1e-300)))
    return np.maximum.reduce(ks)


def sum_grad_scale(name, om, th, sdata):
    """Scale of each summed gradient component: sum_i |d ln P_i / d theta_j|,
    and for the amplitude workloads the per-event bounds summed, sum_i k_i
    (|d_ij| + mean_i |d_ij|) with k_i the amplitude condition number, plus
    n |d ln N / d theta_j| of the amplitude node (its rounding enters once
    per event whatever the events' terms cancel)."""
    _, rows = om.logpdf(th, sdata, grad_rows=True)
    if name not in AMP_WORKLOADS:
        return np.abs(rows).sum(axis=0)
    k = amp_condition(om, th, sdata, name)
    sc = (k[:, None] * (np.abs(rows) + np.abs(rows).mean(axis=0))).sum(axis=0)
    nid, _ = om.dalitz_node()
    return sc + rows.shape[0] * np.abs(om.node_lnnorm(nid, th)[1])


def perturbed_theta(model, spec_, rel=0.5, seed=0):
    """Truth moved by rel x (parameter step) x N(0, 1), kept inside the bounds."""
    rng = np.random.default_rng(seed)
    th = model.theta(spec_["truth"])
    steps = np.array([p[2] for p in spec_["params"]])
    th = th + rel * steps * rng.standard_normal(th.size)
    for i, p in enumerate(spec_["params"]):
        if p[3] != p[4]:
            th[i] = min(max(th[i], p[3] + 1e-9), p[4] - 1e-9)
    return th


def fmt(x):
    return np.array2string(np.asarray(x), precision=3)


def rel_err(a, b, scale):
    return abs(a - b) / scale


def sigma_dev(a, b, sig):
    return np.max(np.abs((np.asarray(a) - np.asarray(b)) / np.asarray(sig)))


def inf_like(x):
    return math.isinf(x)
