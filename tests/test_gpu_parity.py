"""GPU parity: the HIP path (through the C ABI) against the oracle, element
by element on the same seeded events.

Tolerances (stated for every result):
  * NLL: relative 1e-12 (FP64 path) / 1e-6 (FP32-eval path) of
    max(|NLL|, sum_i |ln P_i|);
  * gradient component j: the same relative tolerance of sum_i |d_j ln P_i|;
  * fitted parameters: within 1e-3 sigma of the oracle's fit.
Sizes span many rows (a row is a block's equal share of the 256-event chunks)
and a ragged tail; the row-geometry test adds sizes at chunk boundaries and
one whose rows hold full groups of 8 chunks plus a remainder."""
import math

import numpy as np
import pytest

from helpers import gen_data, get_spec, grad_scale, nll_scale, oracle_for, perturbed_theta, stored_values

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}

CASES = [
    ("c1", 100_123, 11),
    ("c2", 200_077, 12),
    ("listing2", 50_005, 13),
    ("poly", 30_003, 14),
    ("c3", 20_037, 15),
    ("c4", 20_041, 16),
    ("c4x", 20_043, 17),
    ("mapped", 150_001, 18),
    ("mapped_sum", 150_003, 19),
    ("shared", 100_003, 26),
    ("shared_sum", 100_005, 27),
    ("shared_2d", 100_007, 28),
    ("c4s", 20_047, 29),
    ("conv", 50_021, 30),
    ("conv_poly", 50_023, 31),
    ("comp", 50_027, 33),
    ("conv_gmix", 50_029, 35),
]


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


_data_cache = {}


def data_for(name, n, seed):
    key = (name, n, seed)
    if key not in _data_cache:
        _data_cache[key] = gen_data(name, n, seed)
    return _data_cache[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,n,seed", CASES)
def test_nll_and_gradient_match_oracle(P, stream, name, n, seed, prec):
    print(f"\n[case] {name} n={n} prec={prec}", flush=True)
    sp = get_spec(name)
    data = data_for(name, n, seed)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    free = g.free_mask()
    tol = TOL[prec]
    thetas = [om.theta(sp["truth"]), perturbed_theta(om, sp, seed=seed + 1), om.theta()]
    # the oracle evaluates the events as the dataset stores them (FP32-eval:
    # float offsets from the column references)
    sdata = stored_values(sp, data, prec)
    for k, th in enumerate(thetas):
        v_ref, g_ref = om.nll(th, sdata, grad=True)
        v, gr = P.nll_grad(g, ds, th, stream)
        v_only = P.nll_eval(g, ds, th, stream)
        s = nll_scale(om, th, sdata)
        gs = grad_scale(om, th, sdata)
        print(f"  theta#{k}: nll {v:.10g} ref {v_ref:.10g} rel {abs(v - v_ref) / s:.2e}; "
              f"grad rel max {np.max(np.abs(gr - g_ref)[free] / gs[free]):.2e}", flush=True)
        assert abs(v - v_ref) <= tol * s
        assert abs(v_only - v_ref) <= tol * s
        assert np.all(np.abs(gr - g_ref)[free] <= tol * gs[free])
        # bitwise reproducible
        v2, gr2 = P.nll_grad(g, ds, th, stream)
        assert v2 == v and np.array_equal(gr2, gr)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4s", "mapped", "comp", "conv", "conv_gmix"])
def test_batched_equals_single_bitwise(P, stream, name, prec):
    print(f"\n[case] batched {name} {prec}", flush=True)
    sp = get_spec(name)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    sizes = [5_003, 37, 12_345] if name not in ("c3", "c4s") else [1_501, 37, 3_000]
    dss, ths = [], []
    for i, n in enumerate(sizes):
        d = data_for(name, n, 100 + i)
        dss.append(P.Dataset(g, d, prec, stream))
        ths.append(perturbed_theta(om, sp, seed=10 + i))
    datas = [data_for(name, n, 100 + i) for i, n in enumerate(sizes)]
    sizes_all = sizes + [sizes[0]]
    # the first dataset again at another parameter point: a repeated handle
    dss.append(dss[0])
    datas.append(datas[0])
    ths.append(perturbed_theta(om, sp, seed=20))
    nll_b, grad_b = P.nll_grad_batched(g, dss, ths, stream)
    free = g.free_mask()
    for i in range(len(dss)):
        v, gr = P.nll_grad(g, dss[i], ths[i], stream)
        assert v == nll_b[i], (i, v, nll_b[i])
        assert np.array_equal(gr, grad_b[i])
        # and each batched result against the oracle on its own events; the
        # FP32-eval bounds are relative to sums over events and hold once
        # the per-event float rounding averages out (at 37 events the
        # gradient error reaches 3e-6 of its scale), so tiny FP32 datasets
        # are left to the per-event comparison of the terms tests
        if prec == "fp32" and sizes_all[i] < 1000:
            continue
        sd = stored_values(sp, datas[i], prec)
        v_ref, g_ref = om.nll(ths[i], sd, grad=True)
        s = nll_scale(om, ths[i], sd)
        gs = grad_scale(om, ths[i], sd)
        assert abs(nll_b[i] - v_ref) <= TOL[prec] * s, (i, nll_b[i], v_ref)
        assert np.all(np.abs(grad_b[i] - g_ref)[free] <= TOL[prec] * gs[free]), i
    assert nll_b[0] != nll_b[-1]
    # the same fit alone in a batch of one
    n1, g1 = P.nll_grad_batched(g, dss[1:2], ths[1:2], stream)
    assert n1[0] == nll_b[1] and np.array_equal(g1[0], grad_b[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 4 * 2048 + 1, 2_621_440 + 129])
def test_row_geometry_edges(P, stream, n, prec):
    """Single events, partial and exact chunks, one partial chunk after many
    rows, and 2.6e6 events (rows of 10 chunks: one full group of 8 with the
    next group's loads in flight, then a remainder with the ragged chunk)."""
    print(f"\n[case] row geometry c2 n={n} prec={prec}", flush=True)
    sp = get_spec("c2")
    data = data_for("c2", n, 40 + n % 97)
    om = oracle_for("c2")
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    free = g.free_mask()
    th = perturbed_theta(om, sp, seed=41)
    sdata = stored_values(sp, data, prec)
    v_ref, g_ref = om.nll(th, sdata, grad=True)
    v, gr = P.nll_grad(g, ds, th, stream)
    s = nll_scale(om, th, sdata)
    gs = grad_scale(om, th, sdata)
    print(f"  nll rel {abs(v - v_ref) / s:.2e}; grad rel max {np.max(np.abs(gr - g_ref)[free] / gs[free]):.2e}",
          flush=True)
    assert abs(v - v_ref) <= TOL[prec] * s
    assert np.all(np.abs(gr - g_ref)[free] <= TOL[prec] * gs[free])


def test_empty_and_domain_errors(P, stream):
    sp = get_spec("c1")
    g = P.Graph.from_spec(sp)
    ds0 = P.Dataset(g, {"x": np.zeros(0)}, "fp64", stream)
    v, gr = P.nll_grad(g, ds0, [-0.5], stream)
    assert v == 0.0 and gr[0] == 0.0
    with pytest.raises(P.HipfitError) as ei:
        P.Dataset(g, {"x": np.array([1.0, 10.5])}, "fp64", stream)
    assert ei.value.code == -6
    g2 = P.Graph.from_spec(get_spec("c2"))
    ds2 = P.Dataset(g2, data_for("c2", 5000, 3), "fp32", stream)
    v = P.nll_eval(g2, ds2, [0.3, 5.28, -0.001, -2.0], stream)  # sigma < 0: outside the domain
    assert math.isinf(v)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,n,seed", [("c1", 100_123, 21), ("c2", 200_077, 22), ("listing2", 50_005, 23),
                                         ("mapped", 200_011, 24)])
def test_fit_matches_oracle_fit(P, stream, name, n, seed, prec):
    print(f"\n[case] fit {name} n={n} prec={prec}", flush=True)
    sp = get_spec(name)
    data = data_for(name, n, seed)
    om = oracle_for(name)
    ref = om.fit(data)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    r = P.fit(g, ds, stream=stream)
    free = g.free_mask()
    dev = np.abs(r["theta"] - ref["theta"])[free] / ref["errors"][free]
    print(f"  status {r['status']} n_eval {r['n_eval']} edm {r['edm']:.2e}; "
          f"max |dtheta|/sigma {dev.max():.2e}; err ratio {np.max(np.abs(r['errors'][free] / ref['errors'][free] - 1)):.2e}",
          flush=True)
    assert r["status"] == "OK"
    assert dev.max() <= 1e-3
    assert np.all(np.abs(r["errors"][free] / ref["errors"][free] - 1) < 1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fit_shared_observable_product_matches_oracle_fit(P, stream, prec):
    """Fit of the Gaussian-times-acceptance plus exponential model, with the
    acceptance fixed (free, its coefficients and the Gaussian's mean and
    width are nearly degenerate): the numerically renormalised product is
    fitted like any other node."""
    from oracle import oracle as O
    print(f"\n[case] fit shared_sum (fixed acceptance) prec={prec}", flush=True)
    sp = get_spec("shared_sum")
    sp["params"] = [(p[0], sp["truth"][p[0]], p[2], p[3], p[4], True) if p[0].startswith("e_a") else p
                    for p in sp["params"]]
    data = data_for("shared_sum", 200_013, 25)
    om = O.Model(sp)
    ref = om.fit(data)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    r = P.fit(g, ds, stream=stream)
    free = g.free_mask()
    dev = np.abs(r["theta"] - ref["theta"])[free] / ref["errors"][free]
    print(f"  status {r['status']} n_eval {r['n_eval']}; max |dtheta|/sigma {dev.max():.2e}", flush=True)
    assert r["status"] == "OK"
    assert dev.max() <= 1e-3
    assert np.all(np.abs(r["errors"][free] / ref["errors"][free] - 1) < 1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tddp_sigma_map_child_order_is_irrelevant(P, stream, prec):
    """The product of the time-dependent density and the sigma_t map, its
    children listed either way round, gives the same bits (the fused kernel
    takes the amplitude node first in both)."""
    import copy
    sp = get_spec("c4s")
    sw = copy.deepcopy(sp)
    sw["model"]["children"] = sw["model"]["children"][::-1]
    data = data_for("c4s", 20_047, 29)
    om = oracle_for("c4s")
    th = perturbed_theta(om, sp, seed=5)
    res = []
    for s_ in (sp, sw):
        g = P.Graph.from_spec(s_)
        ds = P.Dataset(g, data, prec, stream)
        res.append(P.nll_grad(g, ds, th, stream))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tddp_sigma_map_mixed_cells_match_oracle(P, stream, prec):
    """The sigma_t map with an exponential, a quadratic and two Gaussian
    cells (the fused kernel's general path, not the Gaussian selection)."""
    import copy
    from oracle import oracle as O
    print(f"\n[case] c4s mixed cells {prec}", flush=True)
    sp = copy.deepcopy(get_spec("c4s"))
    dm = sp["model"]["children"][1]
    dm["children"][0] = {"op": "exp", "obs": "sigma_t", "par": ["st_mu0"]}
    dm["children"][1] = {"op": "poly", "obs": "sigma_t", "par": ["st_mu1", "st_sg1"], "x0": 0.11}
    sp["params"] = [(p[0], p[1], p[2], 0.0, 0.0, p[5]) if p[0] in ("st_mu0", "st_mu1", "st_sg1") else p
                    for p in sp["params"]]
    # the exponential cell leaves st_sg0 unused
    sp["params"] = [p[:5] + (True,) if p[0] == "st_sg0" else p for p in sp["params"]]
    data = data_for("c4s", 20_047, 29)
    om = O.Model(sp)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    free = g.free_mask()
    sdata = stored_values(sp, data, prec)
    for k, th in enumerate([om.theta(sp["truth"]), perturbed_theta(om, sp, seed=9)]):
        v_ref, g_ref = om.nll(th, sdata, grad=True)
        v, gr = P.nll_grad(g, ds, th, stream)
        s = nll_scale(om, th, sdata)
        gs = grad_scale(om, th, sdata)
        print(f"  theta#{k}: nll rel {abs(v - v_ref) / s:.2e}; grad rel max "
              f"{np.max(np.abs(gr - g_ref)[free] / gs[free]):.2e}", flush=True)
        assert abs(v - v_ref) <= TOL[prec] * s
        assert np.all(np.abs(gr - g_ref)[free] <= TOL[prec] * gs[free])


RES_PARAMS = {"conv": ("r_mu", "r_sigma"), "conv_gmix": ("r_mu1", "r_sg1", "r_mu2", "r_sg2", "r_f")}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["conv", "conv_gmix"])
def test_fit_convolution_matches_oracle_fit(P, stream, name, prec):
    """Fit of the smeared exponential plus background with the resolution
    fixed (an exponential smeared by a Gaussian, or by a mixture of
    Gaussians, is the same exponential away from the box's edges, so the
    resolution is barely constrained by these data; in practice it comes
    from a calibration).  Errors within 1e-3 (FP64) and 3e-3 (FP32-eval) of
    the oracle's: both are central differences of the gradient over a tenth
    of an error, and the two sides' steps differ (the NLL's departure from a
    quadratic over them moves the FP64 errors by up to 5e-4 here); in the
    FP32-eval path the gradient also carries float rounding, about 1e-3 of
    the Hessian at those steps for 10^5 events."""
    from oracle import oracle as O
    print(f"\n[case] fit {name} (fixed resolution) prec={prec}", flush=True)
    sp = get_spec(name)
    rp = RES_PARAMS[name]
    sp["params"] = [p[:5] + (True,) if p[0] in rp else p for p in sp["params"]]
    sp["params"] = [(p[0], sp["truth"][p[0]]) + tuple(p[2:]) if p[0] in rp else p for p in sp["params"]]
    data = data_for(name, 100_019, 32)
    om = O.Model(sp)
    ref = om.fit(data)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    r = P.fit(g, ds, stream=stream)
    free = g.free_mask()
    dev = np.abs(r["theta"] - ref["theta"])[free] / ref["errors"][free]
    er = np.abs(r["errors"][free] / ref["errors"][free] - 1)
    print(f"  status {r['status']} n_eval {r['n_eval']}; max |dtheta|/sigma {dev.max():.2e}; "
          f"errors ratio - 1 {er}", flush=True)
    assert r["status"] == "OK"
    assert dev.max() <= 1e-3
    assert np.all(er < (1e-3 if prec == "fp64" else 3e-3))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fit_composition_matches_oracle_fit(P, stream, prec):
    """Fit of the Gaussian of a quadratic with the shell's width fixed (the
    exponent depends on (1 - mu, a1, a2) / sigma only: one direction of the
    four parameters is flat)."""
    from oracle import oracle as O
    print(f"\n[case] fit comp (fixed shell width) prec={prec}", flush=True)
    sp = get_spec("comp")
    sp["params"] = [p[:5] + (True,) if p[0] == "s_sigma" else p for p in sp["params"]]
    data = data_for("comp", 100_003, 34)
    om = O.Model(sp)
    ref = om.fit(data)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, prec, stream)
    r = P.fit(g, ds, stream=stream)
    free = g.free_mask()
    dev = np.abs(r["theta"] - ref["theta"])[free] / ref["errors"][free]
    print(f"  status {r['status']} n_eval {r['n_eval']}; max |dtheta|/sigma {dev.max():.2e}", flush=True)
    assert r["status"] == "OK"
    assert dev.max() <= 1e-3
    assert np.all(np.abs(r["errors"][free] / ref["errors"][free] - 1) < 1e-3)


def test_numerical_gradient_fit_agrees(P, stream):
    sp = get_spec("c2")
    data = data_for("c2", 200_077, 22)
    g = P.Graph.from_spec(sp)
    ds = P.Dataset(g, data, "fp64", stream)
    ra = P.fit(g, ds, stream=stream)
    rn = P.fit(g, ds, grad_mode="numerical", stream=stream)
    free = g.free_mask()
    assert rn["status"] == "OK"
    assert np.max(np.abs(ra["theta"] - rn["theta"])[free] / ra["errors"][free]) < 1e-3
    assert rn["n_eval"] > ra["n_eval"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_device_borrowed_dataset_equals_uploaded(P, stream, prec):
    """dataset_wrap_device on tensors holding the storage format gives the
    same bits as dataset_upload of the same events."""
    import torch
    print(f"\n[case] borrowed columns c2 {prec}", flush=True)
    sp = get_spec("c2")
    data = data_for("c2", 300_001, 50)
    om = oracle_for("c2")
    g = P.Graph.from_spec(sp)
    up = P.Dataset(g, data, prec, stream)
    if prec == "fp64":
        t = torch.from_numpy(data["x"]).to("cuda")
    else:
        ref = g.column_ref("x", "fp32")
        t = torch.from_numpy((data["x"] - ref).astype(np.float32)).to("cuda")
    torch.cuda.synchronize()
    wr = P.Dataset.from_device(g, {"x": t}, prec)
    th = perturbed_theta(om, sp, seed=51)
    v1, g1 = P.nll_grad(g, up, th, stream)
    v2, g2 = P.nll_grad(g, wr, th, stream)
    assert v1 == v2 and np.array_equal(g1, g2)
    wr.free()
    up.free()
