"""Binned datasets on the GPU (dataset_upload_binned): the binned NLL and
chi^2 metrics and their gradients against the oracle's, element by element on
the same histograms, and binned fits against the oracle's fits.

Tolerances: the metric within 1e-12 (FP64) / 1e-6 (FP32-eval) of its scale
(binned NLL: sum |w ln P|; chi^2: sum (w^2 + (K P)^2) / max(w, 1), the size
of the terms that cancel), gradient component j within the same fraction of
sum_i (|m'_i| + |m''_i|) |d_j ln P_i|, m' and m'' the first and second
derivatives of bin i's term with respect to ln P (the second carries the
rounding of ln P into the gradient: for chi^2 it is ~2 K P, far above m');
fitted parameters within 1e-3 sigma."""
import numpy as np
import pytest

import synthgen as S
from helpers import get_spec, oracle_for, perturbed_theta

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1311_1753_amd as P
    return P


@pytest.fixture(scope="module")
def stream(P):
    import torch
    return torch.cuda.current_stream()


def hist1(x, lo, hi, nb):
    counts, edges = np.histogram(x, bins=nb, range=(lo, hi))
    return {"x": 0.5 * (edges[1:] + edges[:-1])}, counts.astype(np.float64), edges[1] - edges[0]


def histogram(name, seed):
    """(centres, weights, bin volume) of a histogram of the workload's events."""
    if name == "c1":
        return hist1(S.gen_c1(n=200_000, seed=seed)["x"], 0.0, 10.0, 100)
    if name == "c2":
        return hist1(S.gen_c2(n=500_000, seed=seed)["x"], 5.2, 5.3, 1000)
    if name == "poly":
        x = np.random.default_rng(seed).uniform(-1.0, 3.0, 100_000)
        return hist1(x, -1.0, 3.0, 64)
    if name == "listing2":
        d = S.gen_listing2(n=100_000, seed=seed)
        counts, ex, ey = np.histogram2d(d["x"], d["y"], bins=40, range=[[0, 10], [0, 10]])
        cx, cy = 0.5 * (ex[1:] + ex[:-1]), 0.5 * (ey[1:] + ey[:-1])
        X, Y = np.meshgrid(cx, cy, indexing="ij")
        return {"x": X.ravel(), "y": Y.ravel()}, counts.ravel(), (ex[1] - ex[0]) * (ey[1] - ey[0])
    if name == "c3":
        from helpers import gen_data
        d = gen_data("c3", 30_000, seed)
        lo, hi = S.dalitz_box()
        nb = 60
        counts, e1, e2 = np.histogram2d(d["s12"], d["s13"], bins=nb, range=[[lo, hi], [lo, hi]])
        c1, c2 = 0.5 * (e1[1:] + e1[:-1]), 0.5 * (e2[1:] + e2[:-1])
        A, B = np.meshgrid(c1, c2, indexing="ij")
        om = oracle_for("c3")  # membership by the oracle's rule (c = 0: |A|^2 = 1 inside)
        inside = om.dalitz_amp2(np.zeros(len(om.par_names)), A.ravel(), B.ravel()) > 0
        # only bins whose centre is inside the plot (their events are kept)
        return ({"s12": A.ravel()[inside], "s13": B.ravel()[inside]}, counts.ravel()[inside],
                (e1[1] - e1[0]) * (e2[1] - e2[0]))
    if name in ("mapped_sum", "shared_sum", "comp", "conv"):
        from helpers import gen_data
        return hist1(gen_data(name, 100_000, seed)["x"], 0.0, 10.0, 100)
    raise ValueError(name)


def scales(om, th, cen, w, metric, vol):
    lp, gr = om.logpdf(th, cen, grad_rows=True)
    if metric == "bnll":
        s = np.sum(np.abs(w * lp))
        d = np.abs(w)
    else:
        K = w.sum() * vol
        E = K * np.exp(lp)
        s2 = np.maximum(w, 1.0)
        s = np.sum((w * w + E * E) / s2)
        d = np.abs(2.0 * (w - E) * E / s2) + np.abs(2.0 * (w - 2.0 * E) * E / s2)
    return s, np.sum(d[:, None] * np.abs(gr), axis=0)


@pytest.mark.parametrize("metric", ["bnll", "chi2"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1", "c2", "poly", "listing2", "c3", "mapped_sum", "shared_sum", "comp", "conv"])
def test_binned_metric_matches_oracle(P, stream, name, prec, metric):
    print(f"\n[case] binned {name} {metric} {prec}", flush=True)
    sp = get_spec(name)
    om = oracle_for(name)
    cen, w, vol = histogram(name, 70)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset.binned(g, cen, w, vol, metric, prec, stream)
    free = g.free_mask()
    for k, th in enumerate([om.theta(sp["truth"]), perturbed_theta(om, sp, seed=71)]):
        v_ref, g_ref = om.binned(th, cen, w, metric, vol, grad=True)
        v, gr = P.nll_grad(g, ds, th, stream)
        v_only = P.nll_eval(g, ds, th, stream)
        s, gs = scales(om, th, cen, w, metric, vol)
        print(f"  theta#{k}: {v:.10g} ref {v_ref:.10g} rel {abs(v - v_ref) / s:.2e}; "
              f"grad rel max {np.max(np.abs(gr - g_ref)[free] / gs[free]):.2e}", flush=True)
        assert abs(v - v_ref) <= TOL[prec] * s
        assert abs(v_only - v_ref) <= TOL[prec] * s
        assert np.all(np.abs(gr - g_ref)[free] <= TOL[prec] * gs[free])
        v2, gr2 = P.nll_grad(g, ds, th, stream)
        assert v2 == v and np.array_equal(gr2, gr)
    ds.free()


def test_unit_weights_reproduce_the_unbinned_nll(P, stream):
    """Raw events as 'bins' of weight 1: the binned NLL is the NLL."""
    sp = get_spec("c2")
    d = S.gen_c2(n=100_003, seed=72)
    om = oracle_for("c2")
    g = P.Graph.from_spec(sp)
    th = perturbed_theta(om, sp, seed=73)
    ub = P.Dataset(g, d, "fp64", stream)
    bn = P.Dataset.binned(g, d, np.ones(100_003), 1.0, "bnll", "fp64", stream)
    v1, g1 = P.nll_grad(g, ub, th, stream)
    v2, g2 = P.nll_grad(g, bn, th, stream)
    assert abs(v1 - v2) <= 1e-12 * abs(v1)
    assert np.allclose(g1, g2, rtol=1e-10, atol=1e-10 * np.abs(g1).max())


def test_zero_weight_bins_and_rejections(P, stream):
    sp = get_spec("poly")
    g = P.Graph.from_spec(sp)
    cen, w, vol = histogram("poly", 74)
    w[::3] = 0.0
    om = oracle_for("poly")
    th = om.theta(sp["truth"])
    for metric in ("bnll", "chi2"):
        ds = P.Dataset.binned(g, cen, w, vol, metric, "fp64", stream)
        v, gr = P.nll_grad(g, ds, th, stream)
        v_ref, g_ref = om.binned(th, cen, w, metric, vol, grad=True)
        assert abs(v - v_ref) <= 1e-12 * max(abs(v_ref), 1.0) * len(w)
        with pytest.raises(P.HipfitError):
            P.nll_grad_batched(g, [ds], [th], stream)
        ds.free()
    with pytest.raises(P.HipfitError):
        P.Dataset.binned(g, cen, -w, vol, "bnll", "fp64", stream)
    with pytest.raises(P.HipfitError):
        P.Dataset.binned(g, cen, w, 0.0, "chi2", "fp64", stream)


@pytest.mark.parametrize("metric", ["bnll", "chi2"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_binned_fit_matches_oracle_fit(P, stream, metric, prec):
    print(f"\n[case] binned fit c2 {metric} {prec}", flush=True)
    sp = get_spec("c2")
    om = oracle_for("c2")
    cen, w, vol = hist1(S.gen_c2(n=2_000_000, seed=75)["x"], 5.2, 5.3, 1000)
    ref = om.fit(cen, binned={"weights": w, "metric": metric, "volume": vol})
    g = P.Graph.from_spec(sp)
    ds = P.Dataset.binned(g, cen, w, vol, metric, prec, stream)
    r = P.fit(g, ds, stream=stream)
    free = g.free_mask()
    dev = np.abs(r["theta"] - ref["theta"])[free] / ref["errors"][free]
    er = np.max(np.abs(r["errors"][free] / ref["errors"][free] - 1))
    print(f"  status {r['status']} n_eval {r['n_eval']} max |dtheta|/sigma {dev.max():.2e} err ratio-1 {er:.2e}",
          flush=True)
    assert r["status"] == "OK"
    assert dev.max() <= 1e-3
    assert er < (1e-3 if prec == "fp64" else 2e-3)
