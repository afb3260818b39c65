"""Device-side toy generation (dataset_generate) against the reference
generator (oracle/toygen.py, pinned to Philox's published known-answer
vectors and to closed-form CDFs): the same events for the same seed, event by
event, in both storage formats; ragged and empty sizes; the full 10^7-event
benchmark workload on sampled events; and a fit of generated events.

Tolerance per event: the two sides evaluate the same formulas in double with
different libm implementations (log1p / expm1 / erf / erfinv), so values
agree to a few ulps, amplified in a Gaussian's tails by erfinv's slope:
|dx| <= 1e-13 |x| + 64 eps sum_g sqrt(2) sigma_g (sqrt(pi) / 2) exp(z_g^2),
z_g = (x - mu_g) / (sqrt(2) sigma_g).  The mixture choices are integers
decided by the same double comparisons on both sides, so every event comes
from the same component.  The FP32-eval storage holds (float)(x - ref): one
float ulp of that offset is added to the tolerance."""
import copy
import math

import numpy as np
import pytest

import synthgen as S
from oracle import toygen as T

pytestmark = pytest.mark.gpu

MIX3 = {
    "obs": [("x", 0.0, 10.0)],
    "params": [("f1", 0.5, 0.1, 0, 1, False), ("f2", 0.2, 0.1, 0, 1, False), ("m1", 3.0, 0.1, 0, 10, False),
               ("s1", 0.5, 0.1, 0.01, 5, False), ("m2", 7.0, 0.1, 0, 10, False), ("s2", 1.5, 0.1, 0.01, 5, False),
               ("al", -0.3, 0.1, -5, 5, False)],
    "truth": {"f1": 0.5, "f2": 0.2, "m1": 3.0, "s1": 0.5, "m2": 7.0, "s2": 1.5, "al": -0.3},
    "model": {"op": "add", "par": ["f1", "f2"], "children": [
        {"op": "gauss", "obs": "x", "par": ["m1", "s1"]}, {"op": "gauss", "obs": "x", "par": ["m2", "s2"]},
        {"op": "exp", "obs": "x", "par": ["al"]}]},
}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1311_1753_amd as P
    return P


def spec_of(name):
    return copy.deepcopy(MIX3 if name == "mix3" else S.workload(name))


def gaussians(sp, th):
    """(mu, sigma, observable) of every Gaussian leaf."""
    pidx = {p[0]: i for i, p in enumerate(sp["params"])}
    out = []

    def walk(nd):
        if nd["op"] == "gauss":
            out.append((th[pidx[nd["par"][0]]], th[pidx[nd["par"][1]]], nd["obs"]))
        for c in nd.get("children", []):
            walk(c)
    walk(sp["model"])
    return out


def tolerance(sp, th, name, x, ref, fp32):
    tol = 1e-13 * np.abs(x)
    for mu, sg, o in gaussians(sp, th):
        if o == name:
            z2 = np.minimum(((x - mu) / (math.sqrt(2.0) * sg)) ** 2, 700.0)
            tol = tol + 64 * np.finfo(float).eps * math.sqrt(2.0) * sg * (math.sqrt(math.pi) / 2) * np.exp(z2)
    if fp32:
        tol = tol + np.spacing(np.abs(x - ref).astype(np.float32)).astype(np.float64)
    return tol


def check(P, sp, th, n, seed, prec, idx=None):
    g = P.Graph.from_spec(sp)
    ds = P.Dataset.generate(g, th, n, seed, prec)
    assert ds.n == n
    ref = T.generate(sp, th, n, seed, idx=idx)
    worst = 0.0
    for name, xr in ref.items():
        x = ds.column(name)
        if idx is not None:
            x = x[idx]
        r = g.column_ref(name, prec)
        expect = (xr - r).astype(np.float32).astype(np.float64) + r if prec == "fp32" else xr
        tol = tolerance(sp, th, name, xr, r, prec == "fp32")
        lo, hi = [o[1:] for o in sp["obs"] if o[0] == name][0]
        assert np.all(x >= lo - 1e-6 * (hi - lo)) and np.all(x <= hi + 1e-6 * (hi - lo))
        bad = np.abs(x - expect) > tol
        assert not bad.any(), (name, np.nonzero(bad)[0][:5], x[bad][:5], expect[bad][:5])
        worst = max(worst, float(np.max(np.abs(x - expect) / np.maximum(tol, 1e-300))) if x.size else 0.0)
    ds.free()
    return worst


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1", "c2", "listing2", "mix3"])
def test_generated_events_match_reference(P, name, prec):
    sp = spec_of(name)
    th = np.array([sp["truth"][p[0]] for p in sp["params"]])
    for n, seed in [(100_003, 5), (257, (1 << 40) + 3)]:
        print(f"\n[case] toygen {name} n={n} seed={seed} {prec}", flush=True)
        w = check(P, sp, th, n, seed, prec)
        print(f"  worst |dx| / tol {w:.2e}", flush=True)


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257])
def test_generation_edges(P, n):
    print(f"\n[case] toygen c2 n={n}", flush=True)
    sp = spec_of("c2")
    th = np.array([0.3, 5.28, 0.003, -2.0])
    check(P, sp, th, n, 9, "fp64")


def test_events_do_not_depend_on_the_sample_size(P):
    g = P.Graph.from_spec(spec_of("c2"))
    th = [0.3, 5.28, 0.003, -2.0]
    a = P.Dataset.generate(g, th, 1000, 21).column("x")
    b = P.Dataset.generate(g, th, 300_001, 21).column("x")
    assert np.array_equal(a, b[:1000])
    c = P.Dataset.generate(g, th, 1000, 22).column("x")
    assert not np.array_equal(a, c)


def test_full_size_benchmark_workload_sampled(P):
    """10^7 events of the benchmark workload: the first and last 2000 events
    and 2000 spread between them."""
    print("\n[case] toygen c2 full size (sampled)", flush=True)
    sp = spec_of("c2")
    th = np.array([sp["truth"][p[0]] for p in sp["params"]])
    n = S.C2["n_events"]
    idx = np.unique(np.concatenate([np.arange(2000), np.arange(n - 2000, n),
                                    np.random.default_rng(3).integers(0, n, 2000)]))
    for prec in ("fp64", "fp32"):
        w = check(P, sp, th, n, 2024, prec, idx=idx)
        print(f"  {prec}: worst |dx| / tol {w:.2e}", flush=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fit_of_generated_toy_recovers_truth(P, prec):
    """A generated C1 toy fitted on the device: the estimate lies within 4
    sigma of the truth, and equals the fit of the same events uploaded from
    the host."""
    sp = spec_of("c1")
    g = P.Graph.from_spec(sp)
    ds = P.Dataset.generate(g, [-0.5], 100_000, 77, prec)
    r = P.fit(g, ds)
    assert r["status"] == "OK"
    assert abs(r["theta"][0] + 0.5) < 4 * r["errors"][0]
    up = P.Dataset(g, {"x": ds.column("x")}, prec)
    r2 = P.fit(g, up)
    assert abs(r2["theta"][0] - r["theta"][0]) <= 1e-6 * r["errors"][0]


def _envelope(sp, th, grid=300):
    """1.5 x the oracle's density maximum over a grid of the box."""
    from oracle import oracle as O
    m = O.Model(sp)
    names = [o[0] for o in sp["obs"]]
    axes = [np.linspace(o[1], o[2], grid) for o in sp["obs"]]
    mesh = np.meshgrid(*axes, indexing="ij")
    p = np.exp(m.logpdf(th, {k: v.ravel() for k, v in zip(names, mesh)}))
    return 1.5 * float(np.max(p[np.isfinite(p)]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,n", [("c3", 20_011), ("mapped", 30_001), ("comp", 30_003), ("conv_poly", 5_003)])
def test_accept_reject_events_match_reference(P, name, n, prec):
    """Candidates are the same doubles on both sides (lo + u (hi - lo)), and
    the acceptance u * envelope < P is decided in double on both: the events
    agree exactly, apart from decisions within rounding of a tie (none
    expected at these sizes)."""
    print(f"\n[case] toygen accept-reject {name} n={n} {prec}", flush=True)
    sp = spec_of(name)
    th = np.array([sp["truth"][p[0]] for p in sp["params"]])
    env = _envelope(sp, th, grid=300 if len(sp["obs"]) == 2 else 4001)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset.generate_ar(g, th, n, 99, env, precision=prec)
    ref = T.generate_ar(sp, th, n, 99, env)
    for k, xr in ref.items():
        x = ds.column(k)
        r = g.column_ref(k, prec)
        expect = (xr - r).astype(np.float32).astype(np.float64) + r if prec == "fp32" else xr
        bad = x != expect
        print(f"  {k}: {int(bad.sum())} differing events", flush=True)
        assert bad.sum() == 0


def test_accept_reject_refuses_a_low_envelope(P):
    sp = spec_of("c1")
    g = P.Graph.from_spec(sp)
    with pytest.raises(P.HipfitError) as ei:
        P.Dataset.generate_ar(g, [-0.5], 1000, 1, 0.3)
    assert ei.value.code == -6
    with pytest.raises(P.HipfitError) as ei:
        P.Dataset.generate_ar(g, [-0.5], 1000, 1, 1e6, max_trials=1)
    assert ei.value.code == -6
