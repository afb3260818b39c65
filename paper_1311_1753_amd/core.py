"""Graph / Dataset handles over the C ABI and the likelihood calls.

A `Graph` is a validated PDF tree (pdf_graph_create), a `Dataset` is a set of
events copied to the GPU (dataset_upload).  Trees are given as nested dicts
(the same neutral form the workload descriptions use):

    {"op": "add", "par": ["f"], "children": [
        {"op": "gauss", "obs": "x", "par": ["mu", "sigma"]},
        {"op": "exp", "obs": "x", "par": ["beta"]}]}

with observables [(name, lo, hi)] and parameters
[(name, init, step, lo, hi, fixed)].
"""
import ctypes
import threading

import numpy as np

from . import _lib
from ._lib import check, lib

FP64 = _lib.HF_FP64
FP32_EVAL = _lib.HF_FP32_EVAL
_CH = {"12": 12, "13": 13, "23": 23}


def _stream_ptr(stream):
    """hipStream_t from None / int / torch.cuda.Stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream or None
    ptr = getattr(stream, "cuda_stream", None)
    if ptr is not None:
        return ptr or None
    raise TypeError("stream must be None, an int handle or a torch.cuda.Stream")


def _prec(p):
    if p in (FP64, "fp64", "f64", "double"):
        return FP64
    if p in (FP32_EVAL, "fp32", "f32", "fp32_eval", "float"):
        return FP32_EVAL
    raise ValueError("precision must be 'fp64' or 'fp32'")


def dalitz_consts(dz, node=None):
    """Constant block of a DALITZ / TDDP node (see include/hipfit.h); the
    full time-dependent form (node "qp" set, or resonances with "float")
    appends the flags (1: x, 2: q/p) and the floating-shape flags."""
    res = dz["resonances"]
    c = [dz["M"], dz["m1"], dz["m2"], dz["m3"], dz["r"], float(dz["grid"]), float(len(res))]
    for r in res:
        c += [float(_CH[r["ch"]]), r["m0"], r["g0"], float(r["J"])]
    if node is not None and node["op"] == "tddp" and (node.get("qp") or any(r.get("float") for r in res)):
        c += [float((1 if node.get("x") else 0) | (2 if node.get("qp") else 0))]
        c += [1.0 if r.get("float") else 0.0 for r in res]
    return c


class Graph:
    """A validated, flattened PDF tree living in the library."""

    def __init__(self, obs, params, model):
        self.obs = [tuple(o) for o in obs]
        self.params = [tuple(p) if len(p) == 6 else tuple(p) + (False,) for p in params]
        self.obs_names = [o[0] for o in self.obs]
        self.par_names = [p[0] for p in self.params]
        self.model = model
        nodes = []
        keep = []

        def arr(vals, ct):
            a = (ct * max(len(vals), 1))(*vals)
            keep.append(a)
            return a

        def flatten(node):
            kids = [flatten(c) for c in node.get("children", [])]
            op = node["op"]
            ob = node.get("obs", [])
            ob = [ob] if isinstance(ob, str) else list(ob)
            par = [self.par_names.index(n) for n in node.get("par", [])]
            obs_i = [self.obs_names.index(n) for n in ob]
            consts = []
            if op == "poly":
                consts = [float(node.get("x0", 0.0))]
            elif op in ("dalitz", "tddp"):
                consts = dalitz_consts(node["dalitz"], node)
            elif op == "map":
                consts = [float(b) for b in node["bounds"]]
            elif op == "conv":
                consts = [float(node["grid"]), float(node["d_lo"]), float(node["d_hi"])]
            elif op == "dpmap":
                b12, b13 = [float(b) for b in node["b12"]], [float(b) for b in node["b13"]]
                consts = [len(b12) + 1.0, len(b13) + 1.0] + b12 + b13
            n = _lib.hf_node()
            n.op = _lib.OP[op]
            n.n_child = len(kids)
            n.child = arr(kids, ctypes.c_int32)
            n.n_par = len(par)
            n.par = arr(par, ctypes.c_int32)
            n.n_obs = len(obs_i)
            n.obs = arr(obs_i, ctypes.c_int32)
            n.n_const = len(consts)
            n.consts = arr(consts, ctypes.c_double)
            nodes.append(n)
            return len(nodes) - 1

        root = flatten(model)
        o_arr = (_lib.hf_obs * len(self.obs))(*[_lib.hf_obs(o[0].encode(), o[1], o[2]) for o in self.obs])
        p_arr = (_lib.hf_param * max(len(self.params), 1))(
            *[_lib.hf_param(p[0].encode(), p[1], p[2], p[3], p[4], int(bool(p[5]))) for p in self.params])
        n_arr = (_lib.hf_node * len(nodes))(*nodes)
        h = ctypes.c_void_p()
        check(lib().pdf_graph_create(o_arr, len(self.obs), p_arr, len(self.params), n_arr, len(nodes), root,
                                     ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_spec(cls, spec):
        return cls(spec["obs"], spec["params"], spec["model"])

    @property
    def handle(self):
        return self._h

    @property
    def n_par(self):
        return len(self.params)

    def theta(self, values=None):
        th = np.array([p[1] for p in self.params], dtype=np.float64)
        if values:
            for k, v in values.items():
                th[self.par_names.index(k)] = v
        return th

    def free_mask(self):
        return np.array([not p[5] for p in self.params])

    def column_ref(self, name, precision="fp32"):
        """The reference subtracted from observable `name` in the FP32-eval
        storage (0 for FP64)."""
        r = ctypes.c_double()
        check(lib().hf_column_ref(self.handle, self.obs_names.index(name), _prec(precision), ctypes.byref(r)))
        return r.value

    def dataset_bytes(self, n_events, precision="fp32"):
        """Device bytes a dataset of n_events events of this graph takes
        (dataset_bytes_needed)."""
        b = ctypes.c_int64()
        check(lib().dataset_bytes_needed(self._h, int(n_events), _prec(precision), ctypes.byref(b)))
        return b.value

    def dalitz_inside(self, s12, s13):
        a = np.ascontiguousarray(s12, dtype=np.float64)
        b = np.ascontiguousarray(s13, dtype=np.float64)
        out = np.zeros(a.size, dtype=np.uint8)
        check(lib().hf_dalitz_inside(self._h, 0, a.size, a.ctypes.data_as(_lib._DP), b.ctypes.data_as(_lib._DP),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out.astype(bool)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().pdf_graph_destroy(h)
            except Exception:
                pass
            self._h = None


class Dataset:
    """Events of a graph's observables copied to the GPU (structure of arrays)."""

    def __init__(self, graph, columns, precision="fp64", stream=None):
        self.graph = graph
        self.precision = _prec(precision)
        n = None
        arrs = []
        for name in graph.obs_names:
            if name in columns:
                a = np.ascontiguousarray(columns[name], dtype=np.float64)
            else:
                a = None
            if a is not None:
                if n is None:
                    n = a.size
                elif a.size != n:
                    raise ValueError("columns differ in length")
            arrs.append(a)
        if n is None:
            raise ValueError("no columns")
        arrs = [a if a is not None else np.zeros(n) for a in arrs]
        self._keep = arrs
        ptrs = (_lib._DP * len(arrs))(*[a.ctypes.data_as(_lib._DP) for a in arrs])
        h = ctypes.c_void_p()
        check(lib().dataset_upload(graph.handle, ptrs, n, self.precision, _stream_ptr(stream), ctypes.byref(h)))
        self._keep = None
        self._h = h
        self.n = n

    @classmethod
    def binned(cls, graph, centres, weights, bin_volume, metric="bnll", precision="fp64", stream=None):
        """Binned dataset (dataset_upload_binned): bin centres per observable,
        weights (counts) per bin, equal bins of volume bin_volume; metric
        "bnll" (-sum w ln P) or "chi2" (sum (w - K P)^2 / max(w, 1), K = sum(w)
        x bin volume).  nll_eval / nll_grad / fit then evaluate that metric."""
        self = cls.__new__(cls)
        self.graph = graph
        self.precision = _prec(precision)
        m = {"bnll": _lib.HF_METRIC_BNLL, "chi2": _lib.HF_METRIC_CHI2}[metric]
        w = np.ascontiguousarray(weights, dtype=np.float64)
        n = w.size
        arrs = []
        for name in graph.obs_names:
            a = np.ascontiguousarray(centres[name], dtype=np.float64) if name in centres else np.zeros(n)
            if a.size != n:
                raise ValueError("one centre per bin and observable")
            arrs.append(a)
        ptrs = (_lib._DP * len(arrs))(*[a.ctypes.data_as(_lib._DP) for a in arrs])
        h = ctypes.c_void_p()
        check(lib().dataset_upload_binned(graph.handle, ptrs, w.ctypes.data_as(_lib._DP), n, float(bin_volume), m,
                                          self.precision, _stream_ptr(stream), ctypes.byref(h)))
        self._keep = None
        self._h = h
        self.n = n
        return self

    @classmethod
    def generate(cls, graph, theta, n, seed, precision="fp64", stream=None):
        """Toy dataset drawn on the device (dataset_generate): n events of the
        graph's density at theta, Philox4x32-10 stream keyed by seed."""
        self = cls.__new__(cls)
        self.graph = graph
        self.precision = _prec(precision)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.size != graph.n_par:
            raise ValueError("theta needs one value per parameter")
        h = ctypes.c_void_p()
        check(lib().dataset_generate(graph.handle, th.ctypes.data_as(_lib._DP), int(n),
                                     int(seed) & 0xFFFFFFFFFFFFFFFF, self.precision, _stream_ptr(stream),
                                     ctypes.byref(h)))
        self._keep = None
        self._h = h
        self.n = int(n)
        return self

    @classmethod
    def generate_ar(cls, graph, theta, n, seed, envelope, max_trials=10_000, precision="fp64", stream=None):
        """Accept-reject toy dataset drawn on the device (dataset_generate_ar):
        envelope bounds the normalised density over the box."""
        self = cls.__new__(cls)
        self.graph = graph
        self.precision = _prec(precision)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.size != graph.n_par:
            raise ValueError("theta needs one value per parameter")
        h = ctypes.c_void_p()
        check(lib().dataset_generate_ar(graph.handle, th.ctypes.data_as(_lib._DP), int(n),
                                        int(seed) & 0xFFFFFFFFFFFFFFFF, float(envelope), int(max_trials),
                                        self.precision, _stream_ptr(stream), ctypes.byref(h)))
        self._keep = None
        self._h = h
        self.n = int(n)
        return self

    def column(self, name, stream=None):
        """One observable's stored events as float64 (dataset_read_column)."""
        out = np.empty(self.n)
        check(lib().dataset_read_column(self.handle, self.graph.obs_names.index(name), _stream_ptr(stream),
                                        out.ctypes.data_as(_lib._DP)))
        return out

    @classmethod
    def from_device(cls, graph, columns, precision="fp64"):
        """Borrows device tensors instead of copying (dataset_wrap_device):
        columns maps observable names to contiguous CUDA tensors -- float64
        values for "fp64", float32 offsets value - graph.column_ref(name,
        "fp32") for "fp32".  The tensors are kept referenced by the dataset;
        their values are not validated."""
        self = cls.__new__(cls)
        self.graph = graph
        self.precision = _prec(precision)
        want = "torch.float64" if self.precision == FP64 else "torch.float32"
        n = None
        ptrs = (ctypes.c_void_p * len(graph.obs_names))()
        keep = []
        for i, name in enumerate(graph.obs_names):
            t = columns.get(name)
            if t is None:
                continue
            if str(t.dtype) != want or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
                raise ValueError("column %r must be a contiguous 1-d CUDA tensor of %s" % (name, want))
            if n is None:
                n = t.numel()
            elif t.numel() != n:
                raise ValueError("columns differ in length")
            ptrs[i] = t.data_ptr()
            keep.append(t)
        if n is None:
            raise ValueError("no columns")
        h = ctypes.c_void_p()
        check(lib().dataset_wrap_device(graph.handle, ptrs, n, self.precision, ctypes.byref(h)))
        self._keep = keep
        self._h = h
        self.n = n
        return self

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self):
        return lib().dataset_device_bytes(self._h)

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dataset_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _dp(a):
    return a.ctypes.data_as(_lib._DP)


# Per-thread argument buffers of the evaluation calls, by parameter count:
# theta in, gradient and NLL out, with their addresses taken once (a call
# then costs one copy in and one copy out instead of fresh arrays and
# address look-ups).
_tls = threading.local()


def _io(n):
    bufs = getattr(_tls, "bufs", None)
    if bufs is None:
        bufs = _tls.bufs = {}
    b = bufs.get(n)
    if b is None:
        th, g, out = np.empty(n), np.empty(n), ctypes.c_double()
        b = bufs[n] = (th, th.ctypes.data, g, g.ctypes.data, out, ctypes.byref(out))
    return b


def _theta_in(buf, theta, n):
    a = theta if isinstance(theta, np.ndarray) else np.asarray(theta, dtype=np.float64)
    if a.size != n:
        raise ValueError("theta must have %d entries" % n)
    buf[:] = a.reshape(n)


def nll_eval(graph, ds, theta, stream=None, allow_domain=True):
    """NLL at theta (+inf outside the density's domain when allow_domain)."""
    n = graph.n_par
    th, thp, _, _, out, outp = _io(n)
    _theta_in(th, theta, n)
    rc = lib().nll_eval(graph.handle, ds.handle, thp, _stream_ptr(stream), outp)
    if rc < 0:
        check(rc, allow=(_lib.HF_E_DOMAIN,) if allow_domain else ())
    return out.value


def nll_grad(graph, ds, theta, stream=None, allow_domain=True):
    """(NLL, dNLL/dtheta) at theta from the per-event adjoint kernels."""
    n = graph.n_par
    th, thp, g, gp, out, outp = _io(n)
    _theta_in(th, theta, n)
    rc = lib().nll_grad(graph.handle, ds.handle, thp, _stream_ptr(stream), outp, gp)
    if rc < 0:
        check(rc, allow=(_lib.HF_E_DOMAIN,) if allow_domain else ())
    return out.value, g.copy()


def nll_terms(graph, ds, theta, stream=None, grad=True, allow_domain=True):
    """Per-event ln P_i and (grad) d ln P_i / d theta (n_events x n_par, 0 for
    fixed parameters) from the evaluation kernels, in the dataset's stored
    event order."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != graph.n_par:
        raise ValueError("theta must have %d entries" % graph.n_par)
    lp = np.empty(ds.n)
    rows = np.empty((ds.n, graph.n_par)) if grad else None
    rc = lib().nll_terms(graph.handle, ds.handle, th.ctypes.data, _stream_ptr(stream), lp.ctypes.data,
                         rows.ctypes.data if grad else None)
    if rc < 0:
        check(rc, allow=(_lib.HF_E_DOMAIN,) if allow_domain else ())
    return (lp, rows) if grad else lp


def nll_grad_noalloc(graph, columns, theta, precision="fp64", stream=None, allow_domain=True):
    """nll_grad over device tensors the caller holds (columns as for
    Dataset.from_device) with no device allocation by the library: partial
    sums in its fixed scratch array (nll_grad_noalloc).  Calls on one GPU
    must not overlap."""
    prec = _prec(precision)
    want = "torch.float64" if prec == FP64 else "torch.float32"
    ptrs = (ctypes.c_void_p * len(graph.obs_names))()
    n = None
    for i, name in enumerate(graph.obs_names):
        t = columns.get(name)
        if t is None:
            continue
        if str(t.dtype) != want or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
            raise ValueError("column %r must be a contiguous 1-d CUDA tensor of %s" % (name, want))
        if n is not None and t.numel() != n:
            raise ValueError("columns differ in length")
        n = t.numel()
        ptrs[i] = t.data_ptr()
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != graph.n_par:
        raise ValueError("theta must have %d entries" % graph.n_par)
    out = ctypes.c_double()
    g = np.empty(graph.n_par)
    rc = lib().nll_grad_noalloc(graph.handle, ptrs, n or 0, prec, th.ctypes.data, _stream_ptr(stream),
                                ctypes.byref(out), g.ctypes.data)
    if rc < 0:
        check(rc, allow=(_lib.HF_E_DOMAIN,) if allow_domain else ())
    return out.value, g


def nll_grad_batched(graph, datasets, thetas, stream=None):
    """NLL and gradient of many fits (same graph) in one launch."""
    n = len(datasets)
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(n, graph.n_par))
    hs = (ctypes.c_void_p * n)(*[d.handle.value for d in datasets])
    nll = np.zeros(n)
    g = np.zeros((n, graph.n_par))
    check(lib().nll_grad_batched(graph.handle, hs, n, _dp(th), _stream_ptr(stream), _dp(nll), _dp(g)))
    return nll, g


def fit(graph, ds, theta0=None, grad_mode="analytic", max_iter=500, edm_tol=1e-10, want_errors=True,
        stream=None, param_eps=0.0):
    """Minimise the NLL; returns a dict with theta, errors, cov, nll, edm, n_iter, n_eval, status."""
    th = np.ascontiguousarray(graph.theta() if theta0 is None else theta0, dtype=np.float64).copy()
    err = np.zeros(graph.n_par)
    cov = np.zeros((graph.n_par, graph.n_par))
    o = _lib.hf_fit_opts(max_iter, edm_tol, {"analytic": 0, "numerical": 1}[grad_mode], int(want_errors),
                         param_eps)
    s = _lib.hf_fit_summary()
    rc = lib().fit(graph.handle, ds.handle, ctypes.byref(o), _stream_ptr(stream), _dp(th), _dp(err), _dp(cov),
                   ctypes.byref(s))
    check(rc, allow=(_lib.HF_E_NOT_CONVERGED,))
    return {"theta": th, "errors": err, "cov": cov, "nll": s.nll, "edm": s.edm, "n_iter": s.n_iter,
            "n_eval": s.n_eval, "status": _lib.STATUS_NAMES.get(s.status, str(s.status))}


def minimize(fg, params, x0=None, max_iter=500, edm_tol=1e-10, want_errors=True, f_noise=0.0, param_eps=0.0):
    """The library's minimiser on a Python function fg(x) -> (f, grad).

    params: [(name, init, step, lo, hi, fixed)].  param_eps: relative precision
    with which fg sees x (0: exact).  Runs on the host only."""
    n = len(params)
    p_arr = (_lib.hf_param * max(n, 1))(
        *[_lib.hf_param(p[0].encode(), p[1], p[2], p[3], p[4], int(bool(p[5]) if len(p) > 5 else 0))
          for p in params])
    err_box = []

    def cb(xp, fp, gp, user):
        try:
            x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            f, g = fg(x)
            fp[0] = float(f)
            for i in range(n):
                gp[i] = float(g[i])
            return 0
        except Exception as e:  # reported after the call
            err_box.append(e)
            return 1

    cfun = _lib.FG_FN(cb)
    x = np.zeros(n)
    err = np.zeros(n)
    cov = np.zeros((n, n))
    s = _lib.hf_fit_summary()
    o = _lib.hf_fit_opts(max_iter, edm_tol, 0, int(want_errors), param_eps)
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    rc = lib().hf_minimize(n, p_arr, _dp(x0a) if x0a is not None else None, ctypes.byref(o), f_noise, cfun, None,
                           _dp(x), _dp(err), _dp(cov), ctypes.byref(s))
    if err_box:
        raise err_box[0]
    check(rc, allow=(_lib.HF_E_NOT_CONVERGED, _lib.HF_E_DOMAIN))
    return {"theta": x, "errors": err, "cov": cov, "nll": s.nll, "edm": s.edm, "n_iter": s.n_iter,
            "n_eval": s.n_eval, "status": _lib.STATUS_NAMES.get(s.status, str(s.status))}


def profile(enable=None, every=1):
    """Kernel timing hook: profile(True) resets and starts timing every
    `every`-th evaluation, profile(False) stops; returns (eval_ms, reduce_ms,
    n_timed_calls) accumulated so far."""
    e, r, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    flag = -1 if enable is None else (max(1, int(every)) if enable else 0)
    check(lib().hf_profile(flag, ctypes.byref(e), ctypes.byref(r), ctypes.byref(n)))
    return e.value, r.value, n.value


def version():
    return lib().hf_version().decode()
