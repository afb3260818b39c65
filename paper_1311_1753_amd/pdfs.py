"""User-facing objects in the shape of a GooFit program (paper, section
"GooFit code": create variables, create PDF objects, load data, fit).

    xvar  = Variable("xvar", 0, 10)                      # observable (name, lo, hi)
    alpha = Variable("alpha", -2, 0.1, -10, 10)          # parameter (name, init, step, lo, hi)
    data  = UnbinnedDataSet(xvar)
    for v in values: xvar.value = v; data.addEvent()
    pdf   = ExpPdf("exppdf", xvar, alpha)
    pdf.setData(data)                                     # copies events to the GPU
    FitManager(pdf).fit()                                 # alpha.value / alpha.error updated

PDF objects only describe the tree; the evaluation happens in libhipfit.so.
"""
import numpy as np

from .core import Dataset, Graph, fit as _fit, nll_eval as _nll_eval, nll_grad as _nll_grad


class Variable:
    """Observable: Variable(name, lo, hi).  Parameter: Variable(name, init, step, lo, hi)."""

    def __init__(self, name, *args):
        self.name = name
        if len(args) == 2:
            self.lowerlimit, self.upperlimit = float(args[0]), float(args[1])
            self.value = self.lowerlimit
            self.step = 0.0
            self.is_param = False
        elif len(args) == 4:
            self.value, self.step = float(args[0]), float(args[1])
            self.lowerlimit, self.upperlimit = float(args[2]), float(args[3])
            self.is_param = True
        else:
            raise TypeError("Variable(name, lo, hi) or Variable(name, init, step, lo, hi)")
        self.error = 0.0
        self.fixed = False

    def __repr__(self):
        return "Variable(%s=%g)" % (self.name, self.value)


class UnbinnedDataSet:
    """Rows of observable values; addEvent() appends the variables' current values."""

    def __init__(self, variables):
        self.variables = list(variables) if isinstance(variables, (list, tuple)) else [variables]
        self._rows = []

    def addEvent(self):
        self._rows.append([v.value for v in self.variables])

    def getNumEvents(self):
        return len(self._rows)

    def columns(self):
        a = np.array(self._rows, dtype=np.float64).reshape(len(self._rows), len(self.variables))
        return {v.name: a[:, i].copy() for i, v in enumerate(self.variables)}


class GooPdf:
    """Node of a PDF tree."""

    def __init__(self, name, op, obs=(), params=(), children=(), extra=None):
        self.name = name
        self.op = op
        self.obs = list(obs)
        self.params = list(params)
        self.children = list(children)
        self.extra = dict(extra or {})
        self._graph = None
        self._ds = None

    # ---------------------------------------------------------------- tree
    def _collect(self, obs, params):
        for c in self.children:
            c._collect(obs, params)
        for o in self.obs:
            if all(o is not x for x in obs):
                obs.append(o)
        for p in self.params:
            if all(p is not x for x in params):
                params.append(p)

    def _model(self):
        m = {"op": self.op}
        if self.obs:
            m["obs"] = self.obs[0].name if len(self.obs) == 1 else [o.name for o in self.obs]
        if self.params:
            m["par"] = [p.name for p in self.params]
        if self.children:
            m["children"] = [c._model() for c in self.children]
        m.update(self.extra)
        return m

    def variables(self):
        obs, params = [], []
        self._collect(obs, params)
        return obs, params

    def graph(self):
        if self._graph is None:
            obs, params = self.variables()
            self._graph = Graph([(o.name, o.lowerlimit, o.upperlimit) for o in obs],
                                [(p.name, p.value, p.step, p.lowerlimit, p.upperlimit, p.fixed) for p in params],
                                self._model())
            self._params = params
        return self._graph

    def parameter_values(self):
        self.graph()
        return np.array([p.value for p in self._params])

    # ---------------------------------------------------------------- data
    def setData(self, data, precision="fp64", stream=None):
        """Copies the dataset's events to the GPU (they stay in host memory until now)."""
        g = self.graph()
        cols = data.columns() if isinstance(data, UnbinnedDataSet) else data
        self._ds = Dataset(g, cols, precision, stream)
        return self._ds

    def nll(self, stream=None):
        return _nll_eval(self.graph(), self._ds, self.parameter_values(), stream)

    def nll_grad(self, stream=None):
        return _nll_grad(self.graph(), self._ds, self.parameter_values(), stream)


class ExpPdf(GooPdf):
    def __init__(self, name, x, alpha):
        super().__init__(name, "exp", [x], [alpha])


class GaussianPdf(GooPdf):
    def __init__(self, name, x, mean, sigma):
        super().__init__(name, "gauss", [x], [mean, sigma])


class PolynomialPdf(GooPdf):
    """1 + sum_k a_k (x - x0)^k, k = 1..len(coefficients)."""

    def __init__(self, name, x, coefficients, x0=0.0):
        super().__init__(name, "poly", [x], list(coefficients), extra={"x0": float(x0)})


class AddPdf(GooPdf):
    """sum_j f_j P_j + (1 - sum f_j) P_K with K = len(components) = len(fractions) + 1."""

    def __init__(self, name, fractions, components):
        if len(fractions) != len(components) - 1:
            raise ValueError("AddPdf needs one fraction fewer than components")
        super().__init__(name, "add", [], list(fractions), list(components))


class ProdPdf(GooPdf):
    def __init__(self, name, components):
        super().__init__(name, "prod", [], [], list(components))


class DalitzPdf(GooPdf):
    """|1 + sum c_k A_k|^2 over the Dalitz plot; coefficients = [(re_k, im_k)] Variables."""

    def __init__(self, name, s12, s13, coefficients, kinematics):
        flat = [v for pair in coefficients for v in pair]
        super().__init__(name, "dalitz", [s12, s13], flat, extra={"dalitz": dict(kinematics)})


class TddpPdf(GooPdf):
    """Time-dependent Dalitz density with per-event Gaussian resolution
    (mixing parameters y and, when given, x: the trigonometric terms)."""

    def __init__(self, name, s12, s13, t, sigma_t, coefficients, tau, y, kinematics, x=None):
        flat = [v for pair in coefficients for v in pair] + [tau, y] + ([x] if x is not None else [])
        super().__init__(name, "tddp", [s12, s13, t, sigma_t], flat, extra={"dalitz": dict(kinematics)})


class FitManager:
    """Minimises the PDF's NLL and writes the fitted values and errors back
    into the parameter Variables (the MINUIT role)."""

    def __init__(self, pdf):
        self.pdf = pdf
        self.result = None

    def fit(self, grad_mode="analytic", stream=None, **kw):
        g = self.pdf.graph()
        if self.pdf._ds is None:
            raise RuntimeError("setData() first")
        r = _fit(g, self.pdf._ds, self.pdf.parameter_values(), grad_mode=grad_mode, stream=stream, **kw)
        for p, v, e in zip(self.pdf._params, r["theta"], r["errors"]):
            p.value = float(v)
            p.error = float(e)
        self.result = r
        return r
