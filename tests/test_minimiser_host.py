"""The library's minimiser on the host (hf_minimize): the same state machine
that drives GPU fits, checked on functions whose minima are known."""
import hashlib

import numpy as np
import pytest

import synthgen as S


def test_rosenbrock_unbounded():
    import paper_1311_1753_amd as P

    def fg(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
        return f, g

    r = P.minimize(fg, [("a", -1.2, 0.1, 0, 0, False), ("b", 1.0, 0.1, 0, 0, False)], max_iter=2000)
    assert r["status"] == "OK"
    assert np.allclose(r["theta"], [1.0, 1.0], atol=1e-6)


def test_bounded_and_fixed_parameters():
    import paper_1311_1753_amd as P

    def fg(x):
        f = (x[0] - 0.3) ** 2 * 50 + (x[1] - 2.0) ** 2 + (x[2] + 1.0) ** 2
        return f, np.array([100 * (x[0] - 0.3), 2 * (x[1] - 2.0), 2 * (x[2] + 1.0)])

    r = P.minimize(fg, [("p", 0.9, 0.05, 0.0, 1.0, False), ("q", 0.0, 0.1, 0, 0, True),
                        ("s", 0.0, 0.1, -5.0, 5.0, False)])
    assert r["status"] == "OK"
    # within 1e-4 sigma (the EDM < 1e-10 stop)
    assert abs(r["theta"][0] - 0.3) < 1e-5 and r["theta"][1] == 0.0 and abs(r["theta"][2] + 1.0) < 1e-4
    # errors of f with UP = 0.5: 1/sqrt(f'') = 1/sqrt(100) and 1/sqrt(2)
    assert abs(r["errors"][0] - 0.1) < 1e-6 and abs(r["errors"][2] - 1 / np.sqrt(2)) < 1e-6
    assert r["errors"][1] == 0.0


@pytest.mark.parametrize("name,n", [("c1", 50_000), ("c2", 100_000)])
def test_minimiser_matches_oracle_fit_on_the_oracle_nll(oracle_mod, name, n):
    """The minimiser applied to the oracle's NLL lands within 1e-3 sigma of the
    oracle's own scipy fit, with errors within 1e-3 relative."""
    import paper_1311_1753_amd as P
    spec = S.workload(name)
    m = oracle_mod.Model(spec)
    d = {"c1": S.gen_c1, "c2": S.gen_c2}[name](n=n, seed=31)
    ref = m.fit(d)
    r = P.minimize(lambda x: m.nll(x, d, grad=True), spec["params"])
    assert r["status"] == "OK"
    assert np.max(np.abs(r["theta"] - ref["theta"]) / ref["errors"]) < 1e-3
    assert np.max(np.abs(r["errors"] / ref["errors"] - 1)) < 1e-3


def test_minimiser_tolerates_rounding_noise(oracle_mod):
    """f with 1e-9 relative jitter (far above the EDM target) and a gradient
    with matching jitter: the gradient-based line-search acceptance still
    converges close to the minimum."""
    import paper_1311_1753_amd as P
    spec = S.C2
    m = oracle_mod.Model(spec)
    d = S.gen_c2(n=100_000, seed=32)
    gs = np.abs(m.logpdf(m.theta(spec["truth"]), d, grad_rows=True)[1]).sum(axis=0)

    def jit(x, k):
        h = hashlib.sha256(np.asarray(x).tobytes() + bytes([k])).digest()
        return np.frombuffer(h[:8], dtype=np.uint64)[0] / 2.0**64 * 2 - 1

    def fg(x):
        f, g = m.nll(x, d, grad=True)
        f += 1e-9 * abs(f) * jit(x, 0)
        return f, g + np.array([3e-8 * gs[i] * jit(x, i + 1) for i in range(len(g))])

    ref = m.fit(d)
    r = P.minimize(fg, spec["params"], f_noise=1e-9)
    assert r["status"] == "OK"
    assert np.max(np.abs(r["theta"] - ref["theta"]) / ref["errors"]) < 1e-2
    assert np.max(np.abs(r["errors"] / ref["errors"] - 1)) < 1e-2


@pytest.mark.parametrize("param_eps,ok", [(2.0 ** -24, True), (0.0, False)])
def test_final_hessian_steps_clear_parameter_rounding(param_eps, ok):
    """An evaluation that rounds its parameters to float (as the FP32-eval
    kernels do with constants derived from them): with the parameters' relative
    precision given, the final Hessian's difference steps are large against
    that rounding and the errors of this quadratic come out within 1e-4; with exact
    parameters assumed, 0.1 sigma steps are a few float ulps of x and the
    errors are off by several 1e-4 (deterministic for these inputs)."""
    import paper_1311_1753_amd as P
    c = np.array([1.0, -3.0])
    sig = np.array([1e-5, 2e-5])

    def fg(x):
        xf = np.asarray(x, dtype=np.float32).astype(np.float64)
        r = (xf - c) / sig
        return 0.5 * float(r @ r), r / sig

    r = P.minimize(fg, [("a", 1.0002, 1e-4, 0, 0, False), ("b", -2.9996, 1e-4, 0, 0, False)],
                   param_eps=param_eps)
    assert r["status"] == "OK"
    dev = np.max(np.abs(r["errors"] / sig - 1))
    if ok:
        assert dev < 1e-4
    else:
        assert dev > 3e-4
