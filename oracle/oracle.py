"""Python side of the reference oracle (TEST INFRASTRUCTURE ONLY).

Loads the plain double-precision C++ oracle (``oracle.cpp``) through ctypes,
builds PDF trees from the neutral workload descriptions in ``synthgen``, and
provides an independent maximum-likelihood fit (scipy's L-BFGS-B followed by
Newton polishing with a finite-difference Hessian of the exact gradient).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU library.

Parity pins: every function here is checked in tests/test_oracle_*.py against
closed forms, quadrature, textbook special cases, invariants or statistics.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

KINDS = {"exp": 1, "gauss": 2, "poly": 3, "add": 4, "prod": 5, "dalitz": 6, "tddp": 7, "map": 8, "dpmap": 9, "conv": 10, "comp": 11}
_CH = {"12": 12, "13": 13, "23": 23}


def build(force=True):
    """Compile liboracle.so with g++ (plain -O2, no fast-math, no contraction into fused
    multiply-adds: every expression is evaluated as written; OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        L.om_new.restype = vp
        L.om_new.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        L.om_free.argtypes = [vp]
        L.om_set_root.argtypes = [vp, ctypes.c_int]
        L.om_exp.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.om_gauss.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.om_poly.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ip]
        L.om_add.argtypes = [vp, ctypes.c_int, ip, ip]
        L.om_prod.argtypes = [vp, ctypes.c_int, ip]
        L.om_map.argtypes = [vp, ctypes.c_int, ctypes.c_int, ip, dp]
        L.om_comp.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.om_conv.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double]
        L.om_dpmap.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp]
        L.om_dalitz.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                ip, dp, dp, ip, ip, ip]
        L.om_tddp.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                              ctypes.c_int, ctypes.c_int, ip, dp, dp, ip, ip, ip,
                              ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.om_tddp_full.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                   ctypes.c_int, ctypes.c_int, ip, dp, dp, ip, ip, ip, ip, ip] + [ctypes.c_int] * 5
        L.om_set_direct_norm.argtypes = [vp, ctypes.c_int]
        L.om_res_amp_d.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double, dp]
        L.om_nll.restype = ctypes.c_double
        L.om_nll.argtypes = [vp, dp, ctypes.c_int64, ctypes.POINTER(dp), dp, ctypes.c_int]
        L.om_binned.restype = ctypes.c_double
        L.om_binned.argtypes = [vp, dp, ctypes.c_int64, ctypes.POINTER(dp), dp, ctypes.c_int, ctypes.c_double, dp,
                                ctypes.c_int]
        L.om_logpdf.argtypes = [vp, dp, ctypes.c_int64, ctypes.POINTER(dp), dp, dp, ctypes.c_int]
        L.om_node_lnnorm.restype = ctypes.c_double
        L.om_node_lnnorm.argtypes = [vp, ctypes.c_int, dp, dp]
        L.om_dalitz_matrix.restype = ctypes.c_int
        L.om_dalitz_matrix.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp]
        L.om_dalitz_amp2.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp,
                                     ctypes.c_int, ctypes.c_int]
        L.om_dalitz_cross.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        L.om_dalitz_abs_terms.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp]
        L.om_dalitz_amp.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, dp]
        L.om_tddp_rate.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int]
        L.om_inside.restype = ctypes.c_int
        L.om_inside.argtypes = [dp, ctypes.c_double, ctypes.c_double]
        L.om_res_amp.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, dp]
        for f in ("om_econv", "om_econv_dG"):
            getattr(L, f).restype = ctypes.c_double
            getattr(L, f).argtypes = [ctypes.c_double] * 3
        L.om_econv_osc.argtypes = [ctypes.c_double] * 4 + [dp]
        for f in ("om_erfcx", "om_psi"):
            getattr(L, f).restype = ctypes.c_double
            getattr(L, f).argtypes = [ctypes.c_double]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def n_threads_default():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def tddp_is_full(node):
    """A TDDP node of the full model: complex q/p or floating resonance shapes."""
    return bool(node.get("qp")) or any(r.get("float") for r in node["dalitz"]["resonances"])


def tddp_layout(node):
    """Positions in a full TDDP node's parameter list: 2R coefficients, tau,
    y, x (when node["x"]), |q/p| and arg q/p (when node["qp"]), then m0 and
    Gamma0 of every resonance with "float" set, in resonance order (-1:
    absent)."""
    res = node["dalitz"]["resonances"]
    R = len(res)
    k = 2 * R
    lay = {"tau": k, "y": k + 1}
    k += 2
    lay["x"] = k if node.get("x") else -1
    k += 1 if node.get("x") else 0
    lay["qm"], lay["qa"] = (k, k + 1) if node.get("qp") else (-1, -1)
    k += 2 if node.get("qp") else 0
    lay["m0"], lay["g0"] = [], []
    for r in res:
        if r.get("float"):
            lay["m0"].append(k)
            lay["g0"].append(k + 1)
            k += 2
        else:
            lay["m0"].append(-1)
            lay["g0"].append(-1)
    if len(node["par"]) != k:
        raise ValueError("full TDDP node: %d parameters, expected %d" % (len(node["par"]), k))
    return lay


def kin_array(dz):
    return np.array([dz["M"], dz["m1"], dz["m2"], dz["m3"], dz["r"]], dtype=np.float64)


class Model:
    """A PDF tree built from a workload description (see synthgen.configs)."""

    def __init__(self, spec):
        self.spec = spec
        self.obs_names = [o[0] for o in spec["obs"]]
        self.par_names = [p[0] for p in spec["params"]]
        self.lo = np.array([o[1] for o in spec["obs"]], dtype=np.float64)
        self.hi = np.array([o[2] for o in spec["obs"]], dtype=np.float64)
        L = lib()
        self._h = L.om_new(len(self.obs_names), _dp(self.lo), _dp(self.hi), len(self.par_names))
        self.node_ids = []
        root = self._add(spec["model"])
        L.om_set_root(self._h, root)
        self.root = root

    def _o(self, name):
        return self.obs_names.index(name)

    def _p(self, name):
        return self.par_names.index(name)

    def _add(self, node):
        L = lib()
        op = node["op"]
        if op == "exp":
            nid = L.om_exp(self._h, self._o(node["obs"]), self._p(node["par"][0]))
        elif op == "gauss":
            nid = L.om_gauss(self._h, self._o(node["obs"]), self._p(node["par"][0]), self._p(node["par"][1]))
        elif op == "poly":
            keep, pp = _ip([self._p(n) for n in node["par"]])
            nid = L.om_poly(self._h, self._o(node["obs"]), float(node.get("x0", 0.0)), len(node["par"]), pp)
        elif op == "map":
            kids = [self._add(c) for c in node["children"]]
            kk, kp = _ip(kids)
            b = np.ascontiguousarray(node["bounds"], dtype=np.float64)
            nid = L.om_map(self._h, self._o(node["obs"]), len(kids), kp, _dp(b))
        elif op == "comp":
            # children: core (POLY, its value is the argument), shell
            kids = [self._add(c) for c in node["children"]]
            nid = L.om_comp(self._h, self._o(node["obs"]), kids[0], kids[1])
        elif op == "conv":
            # children: model, resolution (one-observable leaves on obs)
            kids = [self._add(c) for c in node["children"]]
            nid = L.om_conv(self._h, self._o(node["obs"]), kids[0], kids[1], int(node["grid"]),
                            float(node["d_lo"]), float(node["d_hi"]))
        elif op == "dpmap":
            # obs = (s12, s13, u); children row-major over the (s12, s13) cells
            kids = [self._add(c) for c in node["children"]]
            kk, kp = _ip(kids)
            b12 = np.ascontiguousarray(node["b12"], dtype=np.float64)
            b13 = np.ascontiguousarray(node["b13"], dtype=np.float64)
            if len(kids) != (b12.size + 1) * (b13.size + 1):
                raise ValueError("dpmap needs (len(b12) + 1) x (len(b13) + 1) children")
            o = [self._o(n) for n in node["obs"]]
            nid = L.om_dpmap(self._h, o[0], o[1], o[2], b12.size + 1, b13.size + 1, kp,
                             _dp(np.append(b12, 0.0)), _dp(np.append(b13, 0.0)))
        elif op in ("add", "prod"):
            kids = [self._add(c) for c in node["children"]]
            kk, kp = _ip(kids)
            if op == "add":
                fk, fp = _ip([self._p(n) for n in node["par"]])
                nid = L.om_add(self._h, len(kids), kp, fp)
            else:
                nid = L.om_prod(self._h, len(kids), kp)
        elif op in ("dalitz", "tddp"):
            dz = node["dalitz"]
            res = dz["resonances"]
            kin = kin_array(dz)
            ch, chp = _ip([_CH[r["ch"]] for r in res])
            m0 = np.array([r["m0"] for r in res], dtype=np.float64)
            g0 = np.array([r["g0"] for r in res], dtype=np.float64)
            J, Jp = _ip([r["J"] for r in res])
            names = node["par"]
            pre, prep = _ip([self._p(names[2 * k]) for k in range(len(res))])
            pim, pimp = _ip([self._p(names[2 * k + 1]) for k in range(len(res))])
            obs = [self._o(o) for o in node["obs"]]
            if op == "dalitz":
                nid = L.om_dalitz(self._h, obs[0], obs[1], _dp(kin), int(dz["grid"]), len(res), chp,
                                  _dp(m0), _dp(g0), Jp, prep, pimp)
            elif not tddp_is_full(node):
                # parameters: 2R coefficients, tau, y and optionally x
                R = len(res)
                p_x = self._p(names[2 * R + 2]) if len(names) == 2 * R + 3 else -1
                nid = L.om_tddp(self._h, obs[0], obs[1], obs[2], obs[3], _dp(kin), int(dz["grid"]),
                                R, chp, _dp(m0), _dp(g0), Jp, prep, pimp,
                                self._p(names[2 * R]), self._p(names[2 * R + 1]), p_x)
            else:
                lay = tddp_layout(node)
                idx = {k: (self._p(names[v]) if v >= 0 else -1) for k, v in lay.items() if not isinstance(v, list)}
                pm, pmp = _ip([self._p(names[v]) if v >= 0 else -1 for v in lay["m0"]])
                pg, pgp = _ip([self._p(names[v]) if v >= 0 else -1 for v in lay["g0"]])
                nid = L.om_tddp_full(self._h, obs[0], obs[1], obs[2], obs[3], _dp(kin), int(dz["grid"]),
                                     len(res), chp, _dp(m0), _dp(g0), Jp, prep, pimp, pmp, pgp,
                                     idx["tau"], idx["y"], idx["x"], idx["qm"], idx["qa"])
        else:
            raise ValueError(op)
        self.node_ids.append((nid, node))
        return nid

    def __del__(self):
        try:
            lib().om_free(self._h)
        except Exception:
            pass

    # -------------------------------------------------------------- evaluation
    def theta(self, values=None):
        """Parameter vector from a {name: value} dict (defaults: start values)."""
        th = np.array([p[1] for p in self.spec["params"]], dtype=np.float64)
        if values:
            for k, v in values.items():
                th[self._p(k)] = v
        return th

    def _cols(self, data):
        arrs = [np.ascontiguousarray(data[n], dtype=np.float64) for n in self.obs_names]
        n = len(arrs[0])
        ptrs = (ctypes.POINTER(ctypes.c_double) * len(arrs))(*[_dp(a) for a in arrs])
        return arrs, ptrs, n

    def nll(self, theta, data, grad=False, n_threads=None):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        keep, ptrs, n = self._cols(data)
        g = np.zeros(len(self.par_names)) if grad else None
        v = lib().om_nll(self._h, _dp(th), n, ptrs, _dp(g) if grad else None,
                         n_threads or n_threads_default())
        return (v, g) if grad else v

    METRICS = {"bnll": 1, "chi2": 2}

    def binned(self, theta, data, weights, metric, volume, grad=False, n_threads=None):
        """Binned metric over bin centres `data` with weights (counts):
        'bnll' = -sum w ln P, 'chi2' = sum (w - K P)^2 / max(w, 1) with
        K = sum(w) * volume (om_binned)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        keep, ptrs, n = self._cols(data)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.size != n:
            raise ValueError("one weight per bin")
        K = float(w.sum()) * float(volume)
        g = np.zeros(len(self.par_names)) if grad else None
        v = lib().om_binned(self._h, _dp(th), n, ptrs, _dp(w), self.METRICS[metric], K, _dp(g) if grad else None,
                            n_threads or n_threads_default())
        return (v, g) if grad else v

    def objective(self, theta, data, grad=False, binned=None):
        """The unbinned NLL, or the binned metric binned = dict(weights,
        metric, volume)."""
        if binned is None:
            return self.nll(theta, data, grad=grad)
        return self.binned(theta, data, binned["weights"], binned["metric"], binned["volume"], grad=grad)

    def logpdf(self, theta, data, grad_rows=False, n_threads=None):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        keep, ptrs, n = self._cols(data)
        out = np.empty(n)
        gr = np.empty((n, len(self.par_names))) if grad_rows else None
        lib().om_logpdf(self._h, _dp(th), n, ptrs, _dp(out), _dp(gr) if grad_rows else None,
                        n_threads or n_threads_default())
        return (out, gr) if grad_rows else out

    def node_lnnorm(self, node_id, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        d = np.zeros(len(self.par_names))
        v = lib().om_node_lnnorm(self._h, node_id, _dp(th), _dp(d))
        return v, d

    def set_direct_norm(self, on=True):
        """Tests: every TDDP normalisation as the grid sum at theta."""
        lib().om_set_direct_norm(self._h, int(bool(on)))

    def dalitz_node(self):
        for nid, node in self.node_ids:
            if node["op"] in ("dalitz", "tddp"):
                return nid, node
        raise ValueError("no Dalitz node")

    def dalitz_matrix(self, which=0):
        nid, node = self.dalitz_node()
        na = len(node["dalitz"]["resonances"]) + 1
        out = np.zeros(2 * na * na)
        lib().om_dalitz_matrix(self._h, nid, which, _dp(out))
        return (out[0::2] + 1j * out[1::2]).reshape(na, na)

    def dalitz_abs_terms(self, theta, s12, s13):
        """sum_k |c_k A_k| (constant term included) per point, 0 outside the
        plot: with |A| the condition number of the amplitude sum."""
        nid, _ = self.dalitz_node()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        a = np.ascontiguousarray(s12, dtype=np.float64)
        b = np.ascontiguousarray(s13, dtype=np.float64)
        out = np.empty(a.size)
        lib().om_dalitz_abs_terms(self._h, nid, _dp(th), a.size, _dp(a), _dp(b), _dp(out))
        return out

    def dalitz_amp2(self, theta, s12, s13, swapped=False, n_threads=None):
        nid, _ = self.dalitz_node()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        a = np.ascontiguousarray(s12, dtype=np.float64)
        b = np.ascontiguousarray(s13, dtype=np.float64)
        out = np.empty(a.size)
        lib().om_dalitz_amp2(self._h, nid, _dp(th), a.size, _dp(a), _dp(b), _dp(out), int(swapped),
                             n_threads or n_threads_default())
        return out

    def dalitz_cross(self, theta, s12, s13, imag=False):
        """Re(conj(A) Abar) (Im with imag=True) at each point (0 outside the
        Dalitz plot)."""
        nid, _ = self.dalitz_node()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        a = np.ascontiguousarray(s12, dtype=np.float64)
        b = np.ascontiguousarray(s13, dtype=np.float64)
        out = np.empty(a.size)
        lib().om_dalitz_cross(self._h, nid, _dp(th), a.size, _dp(a), _dp(b), _dp(out), int(imag))
        return out

    def dalitz_amp(self, theta, s12, s13):
        """The coherent amplitude sum A(s12, s13) (complex; 0 outside)."""
        nid, _ = self.dalitz_node()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        a = np.ascontiguousarray(s12, dtype=np.float64)
        b = np.ascontiguousarray(s13, dtype=np.float64)
        re, im = np.empty(a.size), np.empty(a.size)
        lib().om_dalitz_amp(self._h, nid, _dp(th), a.size, _dp(a), _dp(b), _dp(re), _dp(im))
        return re + 1j * im

    def tddp_rate(self, theta, s12, s13, t, n_threads=None):
        nid, _ = self.dalitz_node()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        a = np.ascontiguousarray(s12, dtype=np.float64)
        b = np.ascontiguousarray(s13, dtype=np.float64)
        tt = np.ascontiguousarray(t, dtype=np.float64)
        out = np.empty(a.size)
        lib().om_tddp_rate(self._h, nid, _dp(th), a.size, _dp(a), _dp(b), _dp(tt), _dp(out),
                           n_threads or n_threads_default())
        return out

    # -------------------------------------------------------------- fitting
    def bounds(self):
        out = []
        for p in self.spec["params"]:
            lo, hi = p[3], p[4]
            out.append((None, None) if lo == hi else (lo, hi))
        return out

    def free_mask(self):
        return np.array([not p[5] for p in self.spec["params"]])

    def hessian(self, theta, data, steps=None, binned=None):
        """Central finite differences of the exact gradient, symmetrised.

        Default steps: a tenth of each parameter's error, from a first pass
        with 1e-4 of the parameter's step size (the NLL is close to quadratic
        over a fraction of an error, so the difference quotient is its second
        derivative there)."""
        theta = np.asarray(theta, dtype=np.float64)
        n = theta.size
        if steps is None:
            pstep = np.array([p[2] for p in self.spec["params"]])
            H0 = self.hessian(theta, data, steps=1e-4 * np.maximum(pstep, 1e-12), binned=binned)
            d = np.diag(H0)
            steps = np.where(d > 0, 0.1 / np.sqrt(np.abs(d) + 1e-300), 1e-4 * pstep)
        H = np.zeros((n, n))
        for j in range(n):
            h = steps[j]
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            gp = self.objective(tp, data, grad=True, binned=binned)[1]
            gm = self.objective(tm, data, grad=True, binned=binned)[1]
            H[:, j] = (gp - gm) / (2 * h)
        return 0.5 * (H + H.T)

    def fit(self, data, theta0=None, polish_edm=1e-12, max_polish=20, binned=None):
        """Minimise the NLL (or a binned metric); returns dict(theta, errors,
        cov, nll, edm).

        The covariance is 2 up H^-1 with H the Hessian of the objective: up =
        0.5 for likelihoods (errors sqrt(diag(H^-1))), 1 for chi^2."""
        up = 1.0 if binned is not None and binned["metric"] == "chi2" else 0.5
        from scipy.optimize import minimize
        free = self.free_mask()
        th0 = self.theta() if theta0 is None else np.asarray(theta0, dtype=np.float64).copy()
        idx = np.nonzero(free)[0]
        bnds = [self.bounds()[i] for i in idx]
        scale = np.array([self.spec["params"][i][2] for i in idx])

        def f(u):
            th = th0.copy()
            th[idx] = u * scale
            v, g = self.objective(th, data, grad=True, binned=binned)
            if not np.isfinite(v):
                return 1e300, np.zeros_like(u)
            return v, g[idx] * scale

        sb = [((lo / s if lo is not None else None), (hi / s if hi is not None else None))
              for (lo, hi), s in zip(bnds, scale)]
        r = minimize(f, th0[idx] / scale, jac=True, method="L-BFGS-B", bounds=sb,
                     options={"maxiter": 2000, "ftol": 1e-15, "gtol": 1e-10, "maxcor": 30})
        th = th0.copy()
        th[idx] = r.x * scale
        edm = np.inf
        for _ in range(max_polish):
            v, g = self.objective(th, data, grad=True, binned=binned)
            H = self.hessian(th, data, binned=binned)[np.ix_(idx, idx)]
            step = np.linalg.solve(H, g[idx])
            edm = 0.5 * float(g[idx] @ step)
            if edm < polish_edm:
                break
            th[idx] -= step
        v, g = self.objective(th, data, grad=True, binned=binned)
        H = self.hessian(th, data, binned=binned)[np.ix_(idx, idx)]
        cov = 2.0 * up * np.linalg.inv(H)
        err = np.zeros(th.size)
        err[idx] = np.sqrt(np.diag(cov))
        edm = 0.5 * float(g[idx] @ np.linalg.solve(H, g[idx]))
        return {"theta": th, "errors": err, "cov": cov, "nll": v, "edm": edm, "free": idx}


# ---------------------------------------------------------------- building blocks
def inside(dz, s12, s13):
    k = kin_array(dz)
    return bool(lib().om_inside(_dp(k), float(s12), float(s13)))


def res_amp(dz, ch, m0, g0, J, s12, s13):
    """{A, Gamma(s), B_J(q), Z_J, BW} of one resonance."""
    k = kin_array(dz)
    out = np.zeros(7)
    lib().om_res_amp(_dp(k), _CH[ch], m0, g0, J, s12, s13, _dp(out))
    return {"A": out[0] + 1j * out[1], "width": out[2], "B": out[3], "Z": out[4],
            "BW": out[5] + 1j * out[6]}


def res_amp_d(dz, ch, m0, g0, J, s12, s13):
    """One resonance amplitude and its m0 and Gamma0 derivatives (complex)."""
    out = np.zeros(6)
    lib().om_res_amp_d(_dp(kin_array(dz)), _CH[ch], m0, g0, J, s12, s13, _dp(out))
    return complex(out[0], out[1]), complex(out[2], out[3]), complex(out[4], out[5])


def econv(t, G, s):
    return lib().om_econv(t, G, s)


def econv_dG(t, G, s):
    return lib().om_econv_dG(t, G, s)


def econv_osc(t, G, w, s):
    """(Cz, Sz, dCz/dG, dSz/dG, dCz/dw, dSz/dw): the Gaussian-resolution
    convolutions of e^{-G t} cos(w t) and e^{-G t} sin(w t) by quadrature."""
    out = np.empty(6)
    lib().om_econv_osc(t, G, w, s, _dp(out))
    return out


def erfcx(x):
    return lib().om_erfcx(x)


def psi(z):
    return lib().om_psi(z)
