"""Seeded sampling for the synthetic workloads (numpy PCG64 streams).

Only textbook sampling lives here (inverse-CDF of a truncated exponential,
rejection for a truncated normal, uniform boxes, Poisson arrivals).  Where a
sample must follow a model density, the density is a caller-supplied function
and this module only performs the accept-reject bookkeeping.
"""
import math

import numpy as np

from .configs import C1, C2, C4, C5, LISTING2, dalitz_box

__all__ = [
    "truncated_exponential", "truncated_normal", "gen_c1", "gen_c2",
    "gen_listing2", "gen_accept_reject_dalitz", "gen_accept_reject_tddp", "gen_accept_reject_1d",
    "gen_flat_box", "serving_trace", "gen_serving_request",
]


def truncated_exponential(rng, n, alpha, lo, hi):
    """Samples of e^{alpha x} restricted to [lo, hi] by inverting its CDF."""
    u = rng.random(n)
    L = hi - lo
    if alpha == 0.0:
        return lo + u * L
    return lo + np.log1p(u * np.expm1(alpha * L)) / alpha


def truncated_normal(rng, n, mu, sigma, lo, hi):
    """Normal(mu, sigma) samples restricted to [lo, hi] by rejection."""
    out = np.empty(n)
    got = 0
    while got < n:
        need = n - got
        z = rng.normal(mu, sigma, size=int(need * 1.1) + 16)
        z = z[(z >= lo) & (z <= hi)][:need]
        out[got:got + z.size] = z
        got += z.size
    return out


def gen_c1(n=None, seed=None, alpha=None, lo=None, hi=None):
    n = C1["n_events"] if n is None else n
    seed = C1["seed"] if seed is None else seed
    alpha = C1["truth"]["alpha"] if alpha is None else alpha
    _, olo, ohi = C1["obs"][0]
    lo = olo if lo is None else lo
    hi = ohi if hi is None else hi
    rng = np.random.default_rng(seed)
    return {"x": truncated_exponential(rng, n, alpha, lo, hi)}


def gen_c2(n=None, seed=None, truth=None):
    n = C2["n_events"] if n is None else n
    seed = C2["seed"] if seed is None else seed
    t = dict(C2["truth"]) if truth is None else truth
    _, lo, hi = C2["obs"][0]
    rng = np.random.default_rng(seed)
    is_sig = rng.random(n) < t["f"]
    n_sig = int(is_sig.sum())
    x = np.empty(n)
    x[is_sig] = truncated_normal(rng, n_sig, t["mu"], t["sigma"], lo, hi)
    x[~is_sig] = truncated_exponential(rng, n - n_sig, t["beta"], lo, hi)
    return {"x": x}


def gen_listing2(n=None, seed=None):
    n = LISTING2["n_events"] if n is None else n
    seed = LISTING2["seed"] if seed is None else seed
    rng = np.random.default_rng(seed)
    (_, xlo, xhi), (_, ylo, yhi) = LISTING2["obs"]
    tr = LISTING2["truth"]
    return {"x": truncated_exponential(rng, n, tr["alpha_x"], xlo, xhi),
            "y": truncated_exponential(rng, n, tr["alpha_y"], ylo, yhi)}


def gen_flat_box(n, seed, inside):
    """Points uniform over the Dalitz bounding box, kept where inside(s12, s13)."""
    lo, hi = dalitz_box()
    rng = np.random.default_rng(seed)
    s12 = np.empty(n)
    s13 = np.empty(n)
    got = 0
    while got < n:
        m = max(4 * (n - got), 1024)
        a = lo + (hi - lo) * rng.random(m)
        b = lo + (hi - lo) * rng.random(m)
        keep = np.asarray(inside(a, b), dtype=bool)
        a, b = a[keep][:n - got], b[keep][:n - got]
        s12[got:got + a.size] = a
        s13[got:got + a.size] = b
        got += a.size
    return {"s12": s12, "s13": s13}


def gen_accept_reject_dalitz(n, seed, density, envelope, batch=1 << 20):
    """Accept-reject over the bounding box: keep (s12, s13) iff u*envelope < density.

    `density(s12, s13)` must return 0 outside the Dalitz plot.  Raises if an
    accepted density exceeds the envelope (the envelope was too low).
    """
    lo, hi = dalitz_box()
    rng = np.random.default_rng(seed)
    s12 = np.empty(n)
    s13 = np.empty(n)
    got = 0
    while got < n:
        a = lo + (hi - lo) * rng.random(batch)
        b = lo + (hi - lo) * rng.random(batch)
        u = rng.random(batch)
        d = np.asarray(density(a, b))
        if np.any(d > envelope):
            raise ValueError("accept-reject envelope too low")
        keep = u * envelope < d
        a, b = a[keep][:n - got], b[keep][:n - got]
        s12[got:got + a.size] = a
        s13[got:got + a.size] = b
        got += a.size
    return {"s12": s12, "s13": s13}


def gen_accept_reject_1d(n, seed, density, envelope, lo, hi, batch=1 << 20):
    """Accept-reject on [lo, hi] for a caller-supplied density(x) <= envelope."""
    rng = np.random.default_rng(seed)
    out = np.empty(n)
    got = 0
    while got < n:
        x = lo + (hi - lo) * rng.random(batch)
        u = rng.random(batch)
        d = np.asarray(density(x))
        if np.any(d > envelope):
            raise ValueError("accept-reject envelope too low")
        keep = x[u * envelope < d][:n - got]
        out[got:got + keep.size] = keep
        got += keep.size
    return out


def gen_accept_reject_tddp(n, seed, rate, envelope, tau, y, sigma_t_range=None,
                           batch=1 << 20, sigma_t_cells=None):
    """Accept-reject for (s12, s13, t_true), then Gaussian smearing of t.

    Candidates: (s12, s13) uniform over the box, t_true ~ Exp with rate
    (1-|y|)/tau.  `rate(s12, s13, t_true)` is the unsmeared decay rate (0
    outside the Dalitz plot) and must satisfy
    rate <= envelope * exp(-(1-|y|) t / tau).  sigma_t ~ U(range), or with
    sigma_t_cells = (b12, b13, [(mu, sigma) per cell]) a normal truncated to
    the range with the parameters of the event's cell on the grid cut at
    b12 / b13 (cells row-major, s12 index first; a boundary belongs to the
    cell above it); t = t_true + sigma_t * N(0, 1).
    """
    sigma_t_range = C4["sigma_t_range"] if sigma_t_range is None else sigma_t_range
    lo, hi = dalitz_box()
    rng = np.random.default_rng(seed)
    g_env = (1.0 - abs(y)) / tau
    cols = {k: np.empty(n) for k in ("s12", "s13", "t", "sigma_t")}
    got = 0
    while got < n:
        a = lo + (hi - lo) * rng.random(batch)
        b = lo + (hi - lo) * rng.random(batch)
        tt = rng.exponential(1.0 / g_env, batch)
        u = rng.random(batch)
        d = np.asarray(rate(a, b, tt))
        env = envelope * np.exp(-g_env * tt)
        if np.any(d > env):
            raise ValueError("accept-reject envelope too low")
        keep = np.nonzero(u * env < d)[0][:n - got]
        k = keep.size
        if sigma_t_cells is None:
            st = sigma_t_range[0] + (sigma_t_range[1] - sigma_t_range[0]) * rng.random(k)
        else:
            b12, b13, cells = sigma_t_cells
            cell = (np.searchsorted(b12, a[keep], side="right") * (len(b13) + 1)
                    + np.searchsorted(b13, b[keep], side="right"))
            st = np.empty(k)
            for c, (mu, sg) in enumerate(cells):
                idx = np.nonzero(cell == c)[0]
                st[idx] = truncated_normal(rng, idx.size, mu, sg, *sigma_t_range)
        cols["s12"][got:got + k] = a[keep]
        cols["s13"][got:got + k] = b[keep]
        cols["t"][got:got + k] = tt[keep] + st * rng.standard_normal(k)
        cols["sigma_t"][got:got + k] = st
        got += k
    return cols


def serving_trace(n_requests=None, seed=None, rate_hz=None):
    """Request list for the toy-fit stream: event counts log-uniform in
    [1e3, 1e6], true alpha jittered by +-10 %, Poisson arrivals."""
    cfg = C5
    n_requests = cfg["n_requests"] if n_requests is None else n_requests
    seed = cfg["seed"] if seed is None else seed
    rate_hz = cfg["rate_hz"] if rate_hz is None else rate_hz
    rng = np.random.default_rng(seed)
    lo, hi = cfg["n_range"]
    n_ev = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(np.int64)
    a0 = cfg["base"]["truth"]["alpha"]
    alpha = a0 * (1.0 + rng.uniform(-cfg["jitter"], cfg["jitter"], n_requests))
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    arrival = np.cumsum(gaps) - gaps[0]
    return [{"id": i, "n": int(n_ev[i]), "alpha": float(alpha[i]),
             "arrival_s": float(arrival[i])} for i in range(n_requests)]


def gen_serving_request(req):
    """Dataset of one toy fit of the stream (C1 model, seed [5, id])."""
    rng = np.random.default_rng([C5["seed"], req["id"]])
    _, lo, hi = C1["obs"][0]
    return {"x": truncated_exponential(rng, req["n"], req["alpha"], lo, hi)}
