"""Parity at the workloads' full sizes, through the same kernels and launch
shapes the benchmark times: every event is compared (the oracle computes the
full NLL and gradient), plus the fitted parameters of the benchmark workload
(10^7 events) against the oracle's fit.

Full-size Dalitz events: the 10^6-event amplitude workload uses the oracle's
accept-reject sample; the 2x10^6-event time-dependent workload uses points
uniform over the Dalitz plot with exponential decay times smeared by
sigma_t ~ U[0.02, 0.2] (a cheaper sample of the same observables and ranges:
the parity claim does not depend on the event distribution); the workloads
with the trigonometric terms (x free) and with the sigma_t density of the
Dalitz-plot cells reuse that sample.

Bounds: NLL within 1e-12 (FP64) / 1e-6 (FP32-eval) of max(|NLL|, sum |ln P_i|);
gradient component j within the same fraction of sum_i |d_j ln P_i|, and for
the amplitude workloads of the per-event bounds summed (helpers.
sum_grad_scale: the amplitude condition number of each event, which is
large for the few events near a zero of the rate, and n |d ln N / d theta_j|)."""
import numpy as np
import pytest

from helpers import full_data, get_spec, nll_scale, oracle_for, perturbed_theta, stored_values, sum_grad_scale

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1311_1753_amd as P
    return P


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c4x", "c4s"])
def test_full_size_nll_grad(P, name, prec):
    print(f"\n[case] full-size {name} {prec}", flush=True)
    sp = get_spec(name)
    data = full_data(name)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec)
    th = perturbed_theta(om, sp, rel=0.01, seed=3)
    sdata = stored_values(sp, data, prec)  # the events as stored (FP32-eval: float offsets)
    v_ref, g_ref = om.nll(th, sdata, grad=True)
    v, gr = P.nll_grad(g, ds, th)
    s = nll_scale(om, th, sdata)
    gs = sum_grad_scale(name, om, th, sdata)
    free = g.free_mask()
    print(f"  n={ds.n} nll rel {abs(v - v_ref) / s:.2e} grad rel max {np.max(np.abs(gr - g_ref)[free] / gs[free]):.2e}",
          flush=True)
    assert abs(v - v_ref) <= TOL[prec] * s
    assert np.all(np.abs(gr - g_ref)[free] <= TOL[prec] * gs[free])


@pytest.mark.timeout(600)
def test_full_size_fit_of_benchmark_workload(P):
    """10^7-event composite fit: FP32-eval and FP64 fits within 1e-3 sigma of the oracle's."""
    print("\n[case] full-size fit c2", flush=True)
    sp = get_spec("c2")
    data = full_data("c2")
    om = oracle_for("c2")
    ref = om.fit(data)
    g = P.Graph.from_spec(sp)
    for prec in ("fp32", "fp64"):
        ds = P.Dataset(g, data, prec)
        r = P.fit(g, ds)
        dev = np.abs(r["theta"] - ref["theta"]) / ref["errors"]
        print(f"  {prec}: status {r['status']} n_eval {r['n_eval']} n_iter {r['n_iter']} edm {r['edm']:.2e} "
              f"max |dtheta|/sigma {dev.max():.2e} "
              f"err ratio-1 {np.max(np.abs(r['errors'] / ref['errors'] - 1)):.2e}", flush=True)
        assert r["status"] == "OK"
        assert dev.max() <= 1e-3
        assert np.all(np.abs(r["errors"] / ref["errors"] - 1) < 2e-3)
        ds.free()
