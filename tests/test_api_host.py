"""Host-side behaviour of the paper-shaped Python API (no GPU)."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_addevent_worked_example():
    import paper_1311_1753_amd as P
    fx = json.load(open(os.path.join(HERE, "golden", "addevent_worked_example.json")))
    xvar = P.Variable("xvar", 0, 20.79)
    data = P.UnbinnedDataSet(xvar)
    assert data.getNumEvents() == 0
    for i, v in enumerate(fx["assignments"]):
        xvar.value = v
        assert data.getNumEvents() == i   # still the old count until addEvent
        data.addEvent()
    assert list(data.columns()["xvar"]) == fx["expected_events"]


def test_listing1_objects_build_a_graph():
    import paper_1311_1753_amd as P
    fx = json.load(open(os.path.join(HERE, "golden", "addevent_worked_example.json")))["listing1"]
    a = fx["alpha"]
    xvar = P.Variable("xvar", 0, 10)
    alpha = P.Variable("alpha", a["init"], a["step"], a["lo"], a["hi"])
    pdf = P.ExpPdf("exppdf", xvar, alpha)
    g = pdf.graph()
    assert g.n_par == 1 and g.par_names == ["alpha"]
    assert list(pdf.parameter_values()) == [-2.0]


def test_composite_objects_share_variables():
    import paper_1311_1753_amd as P
    x = P.Variable("x", 5.2, 5.3)
    f = P.Variable("f", 0.25, 0.01, 0, 1)
    mu = P.Variable("mu", 5.279, 0.001, 5.2, 5.3)
    s = P.Variable("sigma", 0.0035, 0.0005, 1e-4, 0.05)
    b = P.Variable("beta", -1.5, 0.1, -10, 10)
    pdf = P.AddPdf("sum", [f], [P.GaussianPdf("g", x, mu, s), P.ExpPdf("e", x, b)])
    obs, params = pdf.variables()
    assert [o.name for o in obs] == ["x"]
    assert sorted(p.name for p in params) == ["beta", "f", "mu", "sigma"]
    pdf.graph()
    with pytest.raises(ValueError):
        P.AddPdf("bad", [], [P.ExpPdf("e", x, b), P.ExpPdf("e2", x, b)])
