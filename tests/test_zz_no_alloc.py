"""The no-allocation entry point (nll_grad_noalloc) against nll_grad on a
dataset holding the same events: bitwise equal, and within the oracle
tolerances, on two calls in a row, the second with fewer events (the scratch
array keeps the first call's contents)."""
import numpy as np
import pytest

from helpers import gen_data, get_spec, grad_scale, nll_scale, oracle_for, perturbed_theta, stored_values

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1311_1753_amd as P
    return P


def device_columns(P, g, data, prec):
    import torch
    cols = {}
    for name, v in data.items():
        v = np.asarray(v, dtype=np.float64)
        if prec == "fp64":
            cols[name] = torch.tensor(v, dtype=torch.float64, device="cuda")
        else:
            ref = g.column_ref(name, "fp32")
            cols[name] = torch.tensor((v - ref).astype(np.float32), dtype=torch.float32, device="cuda")
    return cols


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,sizes", [("c2", (200_003, 1_001)), ("c3", (20_011, 3_001)),
                                        ("c4", (20_021, 2_999)), ("mapped_sum", (50_001, 2_049))])
def test_noalloc_equals_nll_grad(P, name, sizes, prec):
    import torch
    print(f"\n[case] noalloc {name} {prec} sizes={sizes}", flush=True)
    sp = get_spec(name)
    om = oracle_for(name)
    g = P.Graph.from_spec(sp)
    stream = torch.cuda.current_stream()
    free = g.free_mask()
    for k, n in enumerate(sizes):
        data = gen_data(name, n, 700 + k)
        th = perturbed_theta(om, sp, seed=71 + k)
        ds = P.Dataset(g, data, prec, stream)  # (also computes a Dalitz grid on its first evaluation)
        v_ref, g_ref = P.nll_grad(g, ds, th, stream)
        cols = device_columns(P, g, data, prec)
        torch.cuda.synchronize()
        v, gr = P.nll_grad_noalloc(g, cols, th, prec, stream)
        print(f"  n={n}: nll {v!r} vs {v_ref!r}", flush=True)
        assert v == v_ref and np.array_equal(gr, g_ref)
        sd = stored_values(sp, data, prec)
        vo, go = om.nll(th, sd, grad=True)
        assert abs(v - vo) <= TOL[prec] * nll_scale(om, th, sd)
        gs = grad_scale(om, th, sd)
        assert np.all(np.abs(gr - go)[free] <= TOL[prec] * gs[free])
        ds.free()
