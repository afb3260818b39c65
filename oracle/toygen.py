"""Reference toy generation (TEST INFRASTRUCTURE ONLY).

What the library's device-side generator must produce, written plainly in
numpy: events of a sampleable PDF tree at given parameters, drawn with the
counter-based Philox4x32-10 generator (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011) from its published
definition.  Only the test suite may import this module; it shares no code
with the GPU library.

Random stream.  Uniform number m (m = 0, 1, ...) of event i under a 64-bit
seed s is taken from one Philox4x32-10 block with counter
(i mod 2^32, i div 2^32, m div 2, 0) and key (s mod 2^32, s div 2^32): words
(w0, w1) for even m, (w2, w3) for odd m, mapped to
u = (floor((w_a 2^32 + w_b) / 2^11) + 1/2) 2^-53, strictly inside (0, 1).

Sampling (the paper's toy studies draw events from the fitted model): a PROD
samples its children in order, each on its own observables; an ADD uses one
uniform to pick a child (the first j with u < f_0 + ... + f_j, the last child
taking the rest) and then samples that child; an EXP leaf on [a, b] inverts
its CDF, x = a + ln(1 + u (e^{alpha (b-a)} - 1)) / alpha (a + u (b - a) for
alpha = 0); a GAUSS leaf inverts the truncated normal CDF,
x = mu + sqrt(2) sigma erfinv(erf(z_a) + u (erf(z_b) - erf(z_a))) with
z = (bound - mu) / (sqrt(2) sigma).  Each leaf uses one uniform.  Values are
clamped to the box against rounding.

Parity pins: tests/test_oracle_toygen.py (published Philox known-answer
vectors, Kolmogorov-Smirnov tests against the closed-form CDFs, mixture
fractions, independence of the factors of a product).
"""
import numpy as np
from scipy import special

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: (n, 4) integers < 2^32; key: (n, 2) or
    (2,) integers < 2^32.  Returns (n, 4) uint64 holding 32-bit words."""
    c = np.array(ctr, dtype=np.uint64).reshape(-1, 4)
    k = np.broadcast_to(np.array(key, dtype=np.uint64), (c.shape[0], 2)).copy()
    c0, c1, c2, c3 = (c[:, j].copy() for j in range(4))
    k0, k1 = k[:, 0].copy(), k[:, 1].copy()
    for r in range(10):
        p0 = _M0 * c0          # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
    return np.stack([c0, c1, c2, c3], axis=1)


def uniforms(idx, seed, m):
    """Uniform number m of the events with indices idx (int64 array)."""
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = np.stack([idx & _MASK, idx >> np.uint64(32), np.full(idx.shape, m // 2, dtype=np.uint64),
                    np.zeros(idx.shape, dtype=np.uint64)], axis=1)
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    w = philox4x32_10(ctr, [s & 0xFFFFFFFF, s >> 32])
    a, b = (w[:, 0], w[:, 1]) if m % 2 == 0 else (w[:, 2], w[:, 3])
    bits = ((a << np.uint64(32)) | b) >> np.uint64(11)
    return (bits.astype(np.float64) + 0.5) * 2.0 ** -53


def _box(spec, name):
    for o in spec["obs"]:
        if o[0] == name:
            return float(o[1]), float(o[2])
    raise KeyError(name)


def generate(spec, theta, n, seed, idx=None):
    """Events of spec's model at parameters theta (dict of observable columns):
    events 0 .. n-1, or those with the indices idx (n is then ignored)."""
    pidx = {p[0]: i for i, p in enumerate(spec["params"])}
    th = np.asarray(theta, dtype=np.float64)
    cols = {}
    idx = np.arange(n, dtype=np.int64) if idx is None else np.asarray(idx, dtype=np.int64)
    n = idx.size
    counter = np.zeros(n, dtype=np.int64)  # next uniform number of each event

    def draw(sel):
        """One uniform for each event in sel (its own next number)."""
        out = np.empty(sel.size)
        for m in np.unique(counter[sel]):
            k = counter[sel] == m
            out[k] = uniforms(idx[sel][k], seed, int(m))
        counter[sel] += 1
        return out

    def leaf(node, sel):
        name = node["obs"]
        a, b = _box(spec, name)
        u = draw(sel)
        if node["op"] == "exp":
            al = th[pidx[node["par"][0]]]
            x = a + u * (b - a) if al == 0.0 else a + np.log1p(u * np.expm1(al * (b - a))) / al
        elif node["op"] == "gauss":
            mu, sg = th[pidx[node["par"][0]]], th[pidx[node["par"][1]]]
            ea, eb = special.erf((a - mu) / (np.sqrt(2.0) * sg)), special.erf((b - mu) / (np.sqrt(2.0) * sg))
            x = mu + np.sqrt(2.0) * sg * special.erfinv(ea + u * (eb - ea))
        else:
            raise ValueError("toy generation: unsupported leaf " + node["op"])
        cols.setdefault(name, np.empty(n))[sel] = np.clip(x, a, b)

    def node_(node, sel):
        op = node["op"]
        if op == "prod":
            for c in node["children"]:
                node_(c, sel)
        elif op == "add":
            u = draw(sel)
            f = [th[pidx[p]] for p in node["par"]]
            cum = np.cumsum(f)
            pick = np.searchsorted(cum, u, side="right")  # first j with u < cum[j]
            pick = np.minimum(pick, len(node["children"]) - 1)
            for j, c in enumerate(node["children"]):
                node_(c, sel[pick == j])
        else:
            leaf(node, sel)

    node_(spec["model"], np.arange(n))
    return cols


def generate_ar(spec, theta, n, seed, envelope, max_trials=10_000, logpdf=None):
    """Accept-reject toys of any model whose observables have finite boxes.

    Event i takes trials j = 0, 1, ...: with C observables (spec order), the
    candidate's coordinate c is lo_c + u_m (hi_c - lo_c) with uniform number
    m = j (C + 1) + c of the event, and the acceptance uniform is number
    j (C + 1) + C; the first trial with u_acc * envelope < P(candidate) is
    the event (P = 0 outside the Dalitz plot).  logpdf(theta, columns) is the
    density (default: the oracle model of spec).  Returns the columns; raises
    when an event exhausts max_trials or P exceeds the envelope."""
    if logpdf is None:
        from oracle import oracle as O
        logpdf = O.Model(spec).logpdf
    names = [o[0] for o in spec["obs"]]
    lo = np.array([float(o[1]) for o in spec["obs"]])
    hi = np.array([float(o[2]) for o in spec["obs"]])
    if not (np.all(np.isfinite(lo)) and np.all(np.isfinite(hi))):
        raise ValueError("accept-reject needs finite boxes")
    C = len(names)
    out = {k: np.empty(n) for k in names}
    pending = np.arange(n, dtype=np.int64)
    for j in range(max_trials):
        if pending.size == 0:
            return out
        cand = {names[c]: lo[c] + uniforms(pending, seed, j * (C + 1) + c) * (hi[c] - lo[c]) for c in range(C)}
        ua = uniforms(pending, seed, j * (C + 1) + C)
        p = np.exp(logpdf(theta, cand))
        if np.any(p > envelope):
            raise ValueError("accept-reject envelope too low")
        acc = ua * envelope < p
        for k in names:
            out[k][pending[acc]] = cand[k][acc]
        pending = pending[~acc]
    if pending.size:
        raise ValueError("accept-reject: trials exhausted")
    return out
