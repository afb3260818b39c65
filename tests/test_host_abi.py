"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function the header declares, and graph validation rejects
malformed trees with HF_E_GRAPH before any GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

import synthgen as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "hipfit.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    txt = "\n".join(ln for ln in txt.splitlines() if not ln.lstrip().startswith("typedef"))
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s+([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_header_symbol():
    from paper_1311_1753_amd import _lib
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_graph_creation_for_every_workload():
    import paper_1311_1753_amd as P
    for name in ("c1", "c2", "c3", "c4", "c4x", "listing2", "mapped", "mapped_sum", "shared", "shared_sum",
                 "shared_2d", "c4s", "conv", "conv_poly", "comp", "conv_gmix"):
        g = P.Graph.from_spec(S.workload(name))
        assert g.n_par == len(S.workload(name)["params"])


def _expect_graph_error(obs, params, model):
    import paper_1311_1753_amd as P
    with pytest.raises(P.HipfitError) as ei:
        P.Graph(obs, params, model)
    assert ei.value.code in (-2, -1), ei.value
    return str(ei.value)


def test_graph_validation_errors():
    obs = [("x", 0.0, 1.0), ("y", 0.0, 1.0)]
    par = [("a", -1.0, 0.1, -5, 5, False), ("b", -1.0, 0.1, -5, 5, False), ("f", 0.5, 0.1, 0, 1, False)]
    ex = {"op": "exp", "obs": "x", "par": ["a"]}
    ey = {"op": "exp", "obs": "y", "par": ["b"]}
    # PROD over a shared observable that is not a group of one-observable
    # leaves: a leaf times a sum on the same observable, and the reverse
    sx = {"op": "add", "par": ["f"], "children": [ex, {"op": "exp", "obs": "x", "par": ["b"]}]}
    _expect_graph_error(obs, par, {"op": "prod", "children": [ex, sx]})
    _expect_graph_error(obs, par, {"op": "prod", "children": [sx, ex]})
    # ... and a PROD of a 2-D product with a leaf on one of its observables
    _expect_graph_error(obs, par, {"op": "prod", "children": [{"op": "prod", "children": [ex, ey]},
                                                               {"op": "gauss", "obs": "y", "par": ["a", "b"]}]})
    # leaves sharing x build (renormalised numerically)
    P_ = __import__("paper_1311_1753_amd")
    P_.Graph(obs, par, {"op": "prod", "children": [ex, {"op": "exp", "obs": "x", "par": ["b"]}]})
    # ADD over different observables
    _expect_graph_error(obs, par, {"op": "add", "par": ["f"], "children": [ex, ey]})
    # ADD with a wrong number of fractions
    _expect_graph_error(obs, par, {"op": "add", "par": [], "children": [ex, dict(ex, par=["b"])]})
    # GAUSS with one parameter
    _expect_graph_error(obs, par, {"op": "gauss", "obs": "x", "par": ["a"]})
    # lo >= hi
    _expect_graph_error([("x", 1.0, 1.0)], par, ex)
    # EXP over an unbounded observable
    _expect_graph_error([("x", 0.0, np.inf)], par, ex)
    # Dalitz resonance below threshold
    bad = S.workload("c3")
    m = dict(bad["model"])
    dz = dict(m["dalitz"])
    dz["resonances"] = [dict(dz["resonances"][0], m0=0.2)] + dz["resonances"][1:]
    m["dalitz"] = dz
    _expect_graph_error(bad["obs"], bad["params"], m)
    # CONV: a grid of one point, an empty residual range, a child that is not a leaf
    cv = S.workload("conv_poly")
    for bad in (dict(cv["model"], grid=1), dict(cv["model"], d_lo=1.0, d_hi=1.0),
                dict(cv["model"], children=[cv["model"]["children"][0], dict(cv["model"], grid=16)])):
        _expect_graph_error(cv["obs"], cv["params"], bad)
    # COMP: a core that is not a polynomial
    cp = S.workload("comp")
    _expect_graph_error(cp["obs"], cp["params"], dict(cp["model"], children=cp["model"]["children"][::-1]))
    # DPMAP: alone (not beside a Dalitz node), wrong child count, boundaries
    # outside the box, a child on another observable
    c4s = S.workload("c4s")
    dm = c4s["model"]["children"][1]
    _expect_graph_error(c4s["obs"], c4s["params"], dm)
    _expect_graph_error(c4s["obs"], c4s["params"], dict(c4s["model"], children=[
        c4s["model"]["children"][0], dict(dm, children=dm["children"][:3])]))
    _expect_graph_error(c4s["obs"], c4s["params"], dict(c4s["model"], children=[
        c4s["model"]["children"][0], dict(dm, b12=[3.5])]))
    _expect_graph_error(c4s["obs"], c4s["params"], dict(c4s["model"], children=[
        c4s["model"]["children"][0], dict(dm, children=dm["children"][:3] + [
            {"op": "exp", "obs": "t", "par": ["st_mu3"]}])]))
    # ... beside a Dalitz node on (s13, s12) instead of (s12, s13)
    _expect_graph_error(c4s["obs"], c4s["params"], dict(c4s["model"], children=[
        c4s["model"]["children"][0], dict(dm, obs=["s13", "s12", "sigma_t"])]))
    # MAP: boundaries not increasing, on the box edge, wrong count, a child
    # that is not a leaf on the MAP's observable
    ga = {"op": "gauss", "obs": "x", "par": ["a", "b"]}
    for b in ([0.6, 0.3], [0.0, 0.5], [0.5, 1.0], [0.5]):
        _expect_graph_error(obs, par, {"op": "map", "obs": "x", "bounds": b, "children": [ex, ga, ex]})
    _expect_graph_error(obs, par, {"op": "map", "obs": "x", "bounds": [0.5], "children": [ex, ey]})
    _expect_graph_error(obs, par, {"op": "map", "obs": "x", "bounds": [0.5], "children": [
        ex, {"op": "add", "par": ["f"], "children": [ex, dict(ex, par=["b"])]}]})


def test_graph_create_raw_abi_errors():
    """Index errors only reachable through the raw ABI (child not earlier, root out of range)."""
    from paper_1311_1753_amd import _lib
    L = _lib.lib()
    obs = (_lib.hf_obs * 1)(_lib.hf_obs(b"x", 0.0, 1.0))
    par = (_lib.hf_param * 1)(_lib.hf_param(b"a", -1.0, 0.1, -5.0, 5.0, 0))
    zero = (ctypes.c_int32 * 1)(0)
    one = (ctypes.c_int32 * 1)(1)
    nodes = (_lib.hf_node * 2)()
    nodes[0].op = 4  # ADD referring to a later node
    nodes[0].n_child = 1
    nodes[0].child = one
    nodes[1].op = 1
    nodes[1].n_par = 1
    nodes[1].par = zero
    nodes[1].n_obs = 1
    nodes[1].obs = zero
    h = ctypes.c_void_p()
    assert L.pdf_graph_create(obs, 1, par, 1, nodes, 2, 0, ctypes.byref(h)) == -2
    assert L.pdf_graph_create(obs, 1, par, 1, nodes, 2, 5, ctypes.byref(h)) == -2
    assert b"root" in L.hf_last_error()
    assert L.last_error_message() == L.hf_last_error()
    # a valid single EXP node through the raw ABI
    assert L.pdf_graph_create(obs, 1, par, 1, ctypes.byref(nodes[1]), 1, 0, ctypes.byref(h)) == 0
    n_obs, n_par = ctypes.c_int32(), ctypes.c_int32()
    assert L.pdf_graph_shape(h, ctypes.byref(n_obs), ctypes.byref(n_par)) == 0
    assert (n_obs.value, n_par.value) == (1, 1)
    L.pdf_graph_destroy(h)


def test_dalitz_membership_matches_oracle_rule(oracle_mod):
    """The library's host Dalitz test and the oracle's agree away from the edge."""
    import paper_1311_1753_amd as P
    g = P.Graph.from_spec(S.C3)
    lo, hi = S.dalitz_box()
    rng = np.random.default_rng(1)
    a = lo + (hi - lo) * rng.random(20000)
    b = lo + (hi - lo) * rng.random(20000)
    mine = g.dalitz_inside(a, b)
    dz = S.C3["model"]["dalitz"]
    ref = np.array([oracle_mod.inside(dz, x, y) for x, y in zip(a, b)])
    assert (mine == ref).all()
    assert 0.4 < mine.mean() < 0.55


def test_toy_generation_refuses_unsampleable_graphs_and_bad_parameters():
    """dataset_generate's checks run on the host before any device work."""
    import paper_1311_1753_amd as P
    for name in ("c3", "mapped", "shared", "poly"):
        sp = S.workload(name) if name != "poly" else {
            "obs": [("x", -1.0, 3.0)], "params": [("a1", 0.2, 0.05, 0, 0, False)],
            "model": {"op": "poly", "obs": "x", "par": ["a1"], "x0": 1.0}}
        g = P.Graph.from_spec(sp)
        with pytest.raises(P.HipfitError) as ei:
            P.Dataset.generate(g, g.theta(sp.get("truth")), 10, 1)
        assert ei.value.code == -2, (name, ei.value)
    ee = {"obs": [("x", 0.0, 1.0)], "params": [("a", -1.0, 0.1, 0, 0, False), ("b", 1.0, 0.1, 0, 0, False)],
          "model": {"op": "prod", "children": [{"op": "exp", "obs": "x", "par": ["a"]},
                                               {"op": "exp", "obs": "x", "par": ["b"]}]}}
    with pytest.raises(P.HipfitError) as ei:
        P.Dataset.generate(P.Graph.from_spec(ee), [-1.0, 1.0], 10, 1)
    assert ei.value.code == -2
    g = P.Graph.from_spec(S.workload("c2"))
    for th in ([0.3, 5.28, -0.003, -2.0], [-0.1, 5.28, 0.003, -2.0], [1.2, 5.28, 0.003, -2.0]):
        with pytest.raises(P.HipfitError) as ei:
            P.Dataset.generate(g, th, 10, 1)
        assert ei.value.code == -6, (th, ei.value)


def test_accept_reject_generation_refuses_on_the_host():
    """dataset_generate_ar: unbounded observables (the time-dependent
    density's t), a non-positive envelope and zero trials are refused before
    any device work."""
    import paper_1311_1753_amd as P
    sp = S.workload("c4")
    g = P.Graph.from_spec(sp)
    with pytest.raises(P.HipfitError) as ei:
        P.Dataset.generate_ar(g, g.theta(sp["truth"]), 10, 1, 1.0)
    assert ei.value.code == -2
    g1 = P.Graph.from_spec(S.workload("c1"))
    for env, trials in ((0.0, 10), (float("inf"), 10), (1.0, 0)):
        with pytest.raises(P.HipfitError) as ei:
            P.Dataset.generate_ar(g1, [-0.5], 10, 1, env, max_trials=trials)
        assert ei.value.code == -1, (env, trials)


def test_dalitz_membership_on_the_boundary_matches_the_oracle(oracle_mod):
    """Points placed on the kinematic boundary and a few ulps either side:
    the library's membership rule (the one the upload validation, the
    normalisation grid and the accept-reject generator share) and the
    oracle's agree point by point, and both include exact boundary points
    and reject points clearly outside."""
    import paper_1311_1753_amd as P
    g = P.Graph.from_spec(S.C3)
    dz = S.C3["model"]["dalitz"]
    M, m1, m2, m3 = dz["M"], dz["m1"], dz["m2"], dz["m3"]
    rng = np.random.default_rng(31)
    s12_all, s13_all = [], []
    lo12, hi12 = (m1 + m2) ** 2, (M - m3) ** 2
    for s12 in np.concatenate([rng.uniform(lo12, hi12, 300), [lo12, hi12]]):
        # s13 limits at this s12 (textbook form, in double)
        rs = np.sqrt(s12)
        E1 = (s12 - m2 * m2 + m1 * m1) / (2 * rs)
        E3 = (M * M - s12 - m3 * m3) / (2 * rs)
        p1 = np.sqrt(max(E1 * E1 - m1 * m1, 0.0))
        p3 = np.sqrt(max(E3 * E3 - m3 * m3, 0.0))
        for edge in ((E1 + E3) ** 2 - (p1 + p3) ** 2, (E1 + E3) ** 2 - (p1 - p3) ** 2):
            v = edge
            for k in range(4):
                v = np.nextafter(v, -np.inf)
            for k in range(9):
                s12_all.append(s12)
                s13_all.append(v)
                v = np.nextafter(v, np.inf)
    s12_all, s13_all = np.array(s12_all), np.array(s13_all)
    # and the mirrored points (the swapped ordering's boundary)
    a = np.concatenate([s12_all, s13_all])
    b = np.concatenate([s13_all, s12_all])
    lib_in = g.dalitz_inside(a, b)
    orc_in = np.array([oracle_mod.inside(dz, x, y) for x, y in zip(a, b)])
    assert np.array_equal(lib_in.astype(bool), orc_in)
    # both sides of the boundary occur among the probes
    assert 0 < orc_in.sum() < orc_in.size


def test_dataset_bytes_needed_argument_checks():
    """The reservation query rejects bad arguments before any device query."""
    import paper_1311_1753_amd as P
    from paper_1311_1753_amd import _lib
    L = _lib.lib()
    g = P.Graph.from_spec(S.C1)
    b = ctypes.c_int64(-7)
    assert L.dataset_bytes_needed(None, 10, 0, ctypes.byref(b)) == -1
    assert L.dataset_bytes_needed(g.handle, -1, 0, ctypes.byref(b)) == -1
    assert L.dataset_bytes_needed(g.handle, 10, 5, ctypes.byref(b)) == -1
    assert L.dataset_bytes_needed(g.handle, 10, 0, None) == -1
    assert b.value == -7


def test_noalloc_argument_checks():
    """nll_grad_noalloc rejects bad arguments on the host, before any GPU
    work: NULL outputs, a negative event count, an unknown precision, a
    convolution graph (its events must be stored sorted) and a Dalitz graph
    whose normalisation grid is not computed yet."""
    import paper_1311_1753_amd as P
    from paper_1311_1753_amd import _lib
    L = _lib.lib()
    g = P.Graph.from_spec(S.workload("c2"))
    th = g.theta()
    v = ctypes.c_double()
    gr = np.zeros(g.n_par)
    cols = (ctypes.c_void_p * 1)()
    assert L.nll_grad_noalloc(g.handle, cols, 0, 0, th.ctypes.data, None, None, gr.ctypes.data) == -1
    assert L.nll_grad_noalloc(g.handle, cols, -1, 0, th.ctypes.data, None, ctypes.byref(v), gr.ctypes.data) == -1
    assert L.nll_grad_noalloc(g.handle, cols, 0, 7, th.ctypes.data, None, ctypes.byref(v), gr.ctypes.data) == -1
    assert L.nll_grad_noalloc(g.handle, None, 5, 0, th.ctypes.data, None, ctypes.byref(v), gr.ctypes.data) == -1
    assert L.nll_grad_noalloc(g.handle, cols, 5, 0, th.ctypes.data, None, ctypes.byref(v), gr.ctypes.data) == -1
    for name, what in (("conv", "convolution"), ("c3", "grid")):
        gc = P.Graph.from_spec(S.workload(name))
        tc = gc.theta()
        gg = np.zeros(gc.n_par)
        rc = L.nll_grad_noalloc(gc.handle, cols, 0, 0, tc.ctypes.data, None, ctypes.byref(v), gg.ctypes.data)
        assert rc == -1 and what in L.hf_last_error().decode(), L.hf_last_error()
