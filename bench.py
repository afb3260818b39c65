"""Benchmark of the unbinned NLL + gradient hot path on one MI355X.

Default workload: the composite Gaussian + exponential model on x in
[5.2, 5.3] (f = 0.3, mu = 5.28, sigma = 0.003, beta = -2), 10^7 synthetic
events, 4 free parameters, FP32 per-event arithmetic with double
compensated accumulation.  A step is one pass of the whole hot path:
parameter staging and normalisation on the host, the per-event evaluation +
adjoint kernel, the two-pass reduction, and the host-side minimiser update
(a BFGS iteration's worth of work is exercised by the fit measurements).

Before the W warm-up steps the evaluation runs untimed for --settle-s
seconds (the GPU's clocks reach their steady state); the timed region then
runs exactly K steps with nothing else in it.  Kernel durations come from a
second, untimed pass over the same evaluations with every launch bracketed
by HIP events (recording the stamps slows the evaluations, so it stays out
of the timed region).

Prints ONE JSON line with the metric (events x NLL+grad evaluations per
second), the roofline of the dominant kernel, the same evaluations on the
plain FP64 path (analytic and central-difference gradients), the serving
stream, and the oracle timed on the host (the headline workload, plus
C1 / C3 / C4 throughput and whole fits beside the GPU's fits).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serving]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (packed); 78.6 without packed instructions
FP64_PEAK_TFLOPS = 78.6

# Algorithmic work per event of one NLL + gradient evaluation, recounted from
# the formulas the kernels evaluate (flops: an FMA counts 2; transcendentals
# -- exp, ln, rcp, sqrt, erfcx -- counted apart), and the bound that applies.
# c3: 3 pair kinematics (q^2, q, 1/s, Zemach factors) ~ 45 flops + 6 T,
# 8 resonances x (width, complex reciprocal, barrier x spin) ~ 15 flops + 1 T,
# coefficient sum 8 x 8, |A|^2, ln, 1/|A|^2, 16-slot adjoint 8 x 8, 17
# accumulations: ~330 flops + 16 T.  c4: amplitudes and swapped amplitudes
# (~2 x 245), |A|^2, |Abar|^2, A* Abar, three Gaussian-convolved decays
# (~15 flops + exp + erfcx each), the rate and ln, an 18-slot adjoint
# (~190 flops): ~700 flops + 35 T; c4x adds the complex convolution
# (~40 flops + 1 T) and an x slot; c4s the event's sigma_t cell density and
# its two slots (~12 flops + 0 T).  conv: per grid term in the residual
# window (about 40 % of the 400 points) ~15 flops + 2 T; conv_poly: 10 % of
# 256 points; conv_gmix: two Gaussian components per term (~25 flops + 2 T)
# over about 60 % of 400 points.  c4f (the full mixing model: 15
# resonances, q/p, two floating shapes): amplitudes and swapped amplitudes
# (2 x (45 + 15 x 15)), coefficient sums (2 x 15 x 8), time factors and rate
# (~100 + 4 T), a 39-slot adjoint (~30 x 20) and the floating-shape
# derivatives (2 x 2 x ~80): ~1800 flops + 40 T per event; its grid
# normalisation (the same evaluation without the time factors at every
# cell inside the plot) runs once per evaluation beside it.
WORK = {
    "c1": {"bound": "hbm"}, "c2": {"bound": "hbm"}, "mapped": {"bound": "hbm"}, "mapped_sum": {"bound": "hbm"},
    "shared": {"bound": "hbm"}, "shared_sum": {"bound": "hbm"}, "c1l": {"bound": "hbm"}, "c2l": {"bound": "hbm"},
    "comp": {"bound": "hbm"},
    "c3": {"bound": "alu", "flops": 330.0}, "c4": {"bound": "alu", "flops": 700.0},
    "c4x": {"bound": "alu", "flops": 740.0}, "c4s": {"bound": "alu", "flops": 712.0},
    "conv": {"bound": "alu", "flops": 160 * 15.0}, "conv_poly": {"bound": "alu", "flops": 26 * 15.0},
    "conv_gmix": {"bound": "alu", "flops": 240 * 25.0}, "c4f": {"bound": "alu", "flops": 1800.0},
}

# HBM traffic of the dominant kernel per launch, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs scaled by a copy-kernel calibration (see
# profiles/k_mix_gauss_exp_1e7_hbm_counters.md); valid only for the kernel
# sources it was measured on (sha256 of KERNEL_SOURCES), else reported as null.
KERNEL_SOURCES = ["paper_1311_1753_amd/csrc/eval_kernels.hip", "paper_1311_1753_amd/csrc/eval_device.h",
                  "paper_1311_1753_amd/csrc/device_common.h", "paper_1311_1753_amd/csrc/internal.h",
                  "paper_1311_1753_amd/csrc/kernels.h"]
MEASURED_TRAFFIC = {"sha256": "2fb9877376d8ad893dcbb536491f82576cf24dbc90434cffda746d01ff5215f1",
                    "bytes_per_launch": 40.35e6}


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return MEASURED_TRAFFIC["bytes_per_launch"] if h.hexdigest() == MEASURED_TRAFFIC["sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-fits", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--settle-s", type=float, default=0.5,
                    help="untimed evaluations for this long before the warm-up steps, so that the "
                         "GPU's clocks are at their steady state (a few steps after idle run ~25%% slower)")
    ap.add_argument("--no-oracle-fits", action="store_true",
                    help="skip the oracle's fit timings on the C1-C4 workloads (part of the CPU leg)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 512 MiB device buffer 5 times (reference for the HBM byte counters)")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c4x", "c4s", "c4f", "mapped", "mapped_sum",
                             "shared", "shared_sum", "conv", "conv_poly", "conv_gmix", "comp", "c1l", "c2l"],
                    help="c2 (default): composite Gauss+exp, the metric's workload; c1 exponential, "
                         "c3 Dalitz amplitude sum, c4 time-dependent Dalitz (c4x with x free: the "
                         "trigonometric terms; c4s times the sigma_t density that varies across "
                         "the plot; c4f the full mixing model: 16 amplitudes, q/p, floating "
                         "resonance shapes), mapped / mapped_sum the piecewise density (alone / "
                         "added to an exponential, 1e7 events), shared / shared_sum a Gaussian times "
                         "an acceptance polynomial on the same observable (alone / added to an "
                         "exponential, 1e7 events), conv / conv_poly numerical convolutions "
                         "(1e6 events), comp a Gaussian of a quadratic (1e6 events), c1l / c2l the c1 / c2 "
                         "models at 2^28 / 10^8 events (beyond the last-level cache): throughput only")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def theta_sequence(truth, k, rng):
    """Parameter points a minimiser would visit near the optimum."""
    t = np.array(truth)
    scale = np.array([2e-4, 2e-6, 2e-6, 2e-3])
    return t + scale * rng.standard_normal((k, t.size))


def time_evals(P, g, ds, thetas, stream, grad=True):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for th in thetas:
        if grad:
            P.nll_grad(g, ds, th, stream)
        else:
            P.nll_eval(g, ds, th, stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def settle(P, g, ds, theta, stream, seconds):
    """Untimed evaluations for `seconds`: the GPU clock settles before the
    warm-up steps and the timed region."""
    import torch
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(50):
            P.nll_grad(g, ds, theta, stream)
        n += 50
    torch.cuda.synchronize()
    return n


def kernel_times(P, g, ds, thetas, stream, grad=True):
    """Average likelihood-kernel and reduction durations over an untimed pass
    of the same evaluations as the timed region, every launch bracketed by
    HIP events that take the dispatch's own start and end stamps
    (hipExtLaunchKernel on the evaluation's stream).  Kept out of the timed
    region: recording the stamps costs the evaluations time."""
    P.profile(True, every=1)
    time_evals(P, g, ds, thetas, stream, grad=grad)
    e_ms, r_ms, cnt = P.profile(False)
    return e_ms / max(cnt, 1), r_ms / max(cnt, 1), cnt


def fit_timing(P, g, ds, stream, mode, reps):
    import torch
    out = []
    res = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = P.fit(g, ds, grad_mode=mode, stream=stream)
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return float(np.median(out)), res


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, data, seconds):
    """The oracle (plain FP64 C++) on a bounded sample: all host threads (the
    reported baseline), then one thread."""
    from oracle import oracle as O
    m = O.Model(spec)
    nt = O.n_threads_default()
    n = min(2_000_000, data["x"].size)
    sample = {"x": np.ascontiguousarray(data["x"][:n])}
    th = m.theta(spec["truth"])

    def rate(threads, budget):
        m.nll(th, sample, grad=True, n_threads=threads)
        reps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget or reps < 2:
            m.nll(th, sample, grad=True, n_threads=threads)
            reps += 1
        el = time.perf_counter() - t0
        return n * reps / el, reps, el

    v, reps, el = rate(nt, seconds)
    v1, reps1, el1 = rate(1, max(2.0, seconds / 4))
    return {"value": v, "unit": "events*NLL+grad evals/s", "cores": nt, "kind": "oracle",
            "sample": "first %d of the 10^7 events, %d NLL+gradient evaluations in %.1f s" % (n, reps, el),
            "one_thread_value": v1, "one_thread_sample": "%d evaluations in %.1f s" % (reps1, el1),
            "cpu_model": _cpu_model()}


def oracle_timing(P, S, stream, fits=True):
    """CPU leg: the oracle (plain FP64 C++, all host threads) on the C1, C3
    and C4 workloads -- NLL + gradient throughput on 10^5 events, and whole
    fits from the workloads' start values -- beside the GPU's fits of the same
    events (FP32-eval and FP64 analytic gradient, FP64 central differences).
    Events: C1 from its generator; C3 / C4 accept-reject on the oracle's
    density (10^5 each, the size of the stored oracle fits)."""
    import torch
    from oracle import oracle as O
    nt = O.n_threads_default()
    out = {"threads": nt, "n_events": 100_000}
    for name in ("c1", "c3", "c4"):
        spec = S.workload(name)
        om = O.Model(spec)
        n = 100_000
        t0 = time.perf_counter()
        if name == "c1":
            data = S.gen_c1(n=n, seed=spec["seed"])
        else:
            th = om.theta(spec["truth"])
            lo, hi = S.dalitz_box()
            c = lo + (np.arange(200) + 0.5) * (hi - lo) / 200
            a, b = np.meshgrid(c, c, indexing="ij")
            if name == "c3":
                env = 1.3 * om.dalitz_amp2(th, a.ravel(), b.ravel()).max()
                data = S.gen_accept_reject_dalitz(n, 31, lambda x, y: om.dalitz_amp2(th, x, y), env, batch=1 << 18)
            else:
                env = 1.3 * (om.dalitz_amp2(th, a.ravel(), b.ravel()) +
                             om.dalitz_amp2(th, a.ravel(), b.ravel(), swapped=True)).max()
                data = S.gen_accept_reject_tddp(n, 41, lambda x, yy, t: om.tddp_rate(th, x, yy, t), env,
                                                th[-2], th[-1], batch=1 << 18)
        gen_s = time.perf_counter() - t0
        th = om.theta(spec["truth"])
        om.nll(th, data, grad=True)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 2.0 or reps < 2:
            om.nll(th, data, grad=True)
            reps += 1
        rate = n * reps / (time.perf_counter() - t0)
        rec = {"oracle_events_evals_per_s": rate, "generation_s": gen_s}
        if fits:
            t0 = time.perf_counter()
            ref = om.fit(data)
            rec["oracle_fit_s"] = time.perf_counter() - t0
            g = P.Graph.from_spec(spec)
            for prec, mode in (("fp32", "analytic"), ("fp64", "analytic"), ("fp64", "numerical")):
                ds = P.Dataset(g, data, prec, stream)
                P.fit(g, ds, grad_mode=mode, stream=stream)  # warm (the Dalitz grid on the first call)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = P.fit(g, ds, grad_mode=mode, stream=stream)
                torch.cuda.synchronize()
                key = "gpu_%s_%s" % (prec, mode)
                rec[key + "_fit_s"] = time.perf_counter() - t0
                free = g.free_mask()
                rec[key + "_max_dtheta_over_sigma"] = float(np.max(np.abs(r["theta"] - ref["theta"])[free] /
                                                                   ref["errors"][free]))
                ds.free()
            rec["oracle_over_gpu_fp32_fit_time"] = rec["oracle_fit_s"] / rec["gpu_fp32_analytic_fit_s"]
        out[name] = rec
        log("oracle %s: %.3g events*evals/s%s" % (name, rate, (", fit %.2f s (GPU FP32 %.4f s)" % (
            rec["oracle_fit_s"], rec["gpu_fp32_analytic_fit_s"])) if fits else ""))
    return out


def serving_bench(P, S, n_req):
    """Toy-fit stream: event counts log-uniform in [1e3, 1e6], Poisson arrivals
    at 200 fits/s; continuous batching (FP32-eval, analytic gradient) against
    one-at-a-time FP64 fits with central-difference gradients."""
    import torch
    reqs = S.serving_trace()[:n_req]
    t0 = time.perf_counter()
    cols = {r["id"]: S.gen_serving_request(r) for r in reqs}
    log("serving: generated %d requests (%d events) in %.1f s" %
        (len(reqs), sum(r["n"] for r in reqs), time.perf_counter() - t0))
    g = P.Graph.from_spec(S.C1)
    colf = lambda r: cols[r["id"]]
    start = lambda r: [-2.0]
    up = torch.cuda.Stream()
    out = {"n_requests": len(reqs), "arrival_rate_hz": S.C5["rate_hz"]}
    srv = P.FitServer(g, "fp32", max_slots=256, hbm_budget_bytes=32 << 30, upload_stream=up)
    res_open, s_open = srv.run(reqs, colf, start, realtime=True)
    res_closed, s_closed = srv.run(reqs, colf, start, realtime=False)
    srv.close()
    out["batched_fp32_open_loop"] = s_open
    out["batched_fp32_closed_loop"] = s_closed
    # the same requests with their toys drawn on the device (dataset_generate)
    # instead of generated on the host and uploaded
    gen = lambda r, st: P.Dataset.generate(g, [r["alpha"]], r["n"], (S.C5["seed"] << 32) | r["id"], "fp32", st)
    srv = P.FitServer(g, "fp32", max_slots=256, hbm_budget_bytes=32 << 30, upload_stream=up)
    _, s_open_d = srv.run(reqs[:1024], None, start, realtime=True, dataset_of=gen)
    _, s_closed_d = srv.run(reqs, None, start, realtime=False, dataset_of=gen)
    srv.close()
    out["batched_fp32_open_loop_device_toys"] = s_open_d
    out["batched_fp32_closed_loop_device_toys"] = s_closed_d
    log("serving (device toys): open p50 %.4f p99 %.4f s; closed %.1f fits/s" %
        (s_open_d["p50_latency_s"], s_open_d["p99_latency_s"], s_closed_d["fits_per_s"]))
    # arrival-rate sweep: the same requests (first 1024) at higher Poisson rates
    sweep = []
    srv = P.FitServer(g, "fp32", max_slots=256, hbm_budget_bytes=32 << 30, upload_stream=up)
    base = S.C5["rate_hz"]
    for rate in (1000.0, 5000.0, 20000.0):
        rq = [dict(r, arrival_s=r["arrival_s"] * base / rate) for r in reqs[:1024]]
        _, sm = srv.run(rq, colf, start, realtime=True)
        sweep.append({"rate_hz": rate, "fits_per_s": sm["fits_per_s"], "p50_latency_s": sm["p50_latency_s"],
                      "p99_latency_s": sm["p99_latency_s"], "n": sm["n"]})
    srv.close()
    out["batched_fp32_rate_sweep"] = sweep
    # the baseline on the same trace: one request at a time, FP64 with
    # central-difference gradients, open loop on the wall clock and closed loop
    _, s_base_open = P.serve_one_at_a_time(g, reqs, colf, start, precision="fp64", grad_mode="numerical",
                                           realtime=True)
    res_base, s_base = P.serve_one_at_a_time(g, reqs, colf, start, precision="fp64", grad_mode="numerical")
    out["one_at_a_time_fp64_numerical_open_loop"] = s_base_open
    out["one_at_a_time_fp64_numerical_closed_loop"] = s_base
    dev = [abs(res_closed[i]["theta"][0] - res_base[i]["theta"][0]) / res_base[i]["errors"][0]
           for i in res_base if i in res_closed]
    out["max_dtheta_over_sigma_batched_vs_baseline"] = float(max(dev)) if dev else None
    out["fits_per_s_ratio_closed_loop"] = s_closed["fits_per_s"] / s_base["fits_per_s"]
    out["p99_ratio_open_loop"] = s_open["p99_latency_s"] / s_base_open["p99_latency_s"]
    log("serving: open p50 %.4f p99 %.4f s (baseline %.4f / %.4f); closed %.1f fits/s (baseline %.1f)" %
        (s_open["p50_latency_s"], s_open["p99_latency_s"], s_base_open["p50_latency_s"],
         s_base_open["p99_latency_s"], s_closed["fits_per_s"], s_base["fits_per_s"]))
    return out


def other_workload(args, P, S, torch, stream):
    """Throughput of the NLL+gradient kernels on one of the other workloads
    (events sampled flat over the Dalitz plot for c3/c4: the evaluation cost
    does not depend on where in the plot the events are)."""
    large = {"c1l": ("c1", 1 << 28), "c2l": ("c2", 10 ** 8)}
    base = large[args.workload][0] if args.workload in large else args.workload
    spec = S.workload(base)
    n = large[args.workload][1] if args.workload in large else spec["n_events"]
    g = P.Graph.from_spec(spec)
    if base == "c1":
        data = S.gen_c1(n=n, seed=spec["seed"])
    elif base == "c2":
        data = S.gen_c2(n=n, seed=spec["seed"])
    elif base in ("mapped", "mapped_sum", "shared", "shared_sum", "conv", "conv_poly", "conv_gmix", "comp"):
        # (conv_poly's density is zero below its first grid point)
        data = {"x": np.random.default_rng(spec["seed"]).uniform(0.1 if base == "conv_poly" else 0.0, 10.0, n)}
    else:
        data = S.gen_flat_box(n, spec["seed"], g.dalitz_inside)
        if args.workload in ("c4", "c4x", "c4s", "c4f"):
            rng = np.random.default_rng(spec["seed"] + 100)
            st = rng.uniform(0.02, 0.2, n)
            data["sigma_t"] = st
            data["t"] = rng.exponential(0.41, n) + st * rng.standard_normal(n)
    truth = g.theta(spec["truth"])
    out = {}
    for prec in ("fp32", "fp64"):
        ds = P.Dataset(g, data, prec, stream)
        settle(P, g, ds, truth, stream, args.settle_s)
        for _ in range(args.warmup):
            P.nll_grad(g, ds, truth, stream)
        k = max(20, args.steps // (1 if args.workload == "c1" else 10))
        if args.workload in large:
            k = max(20, args.steps // 20)
        el = time_evals(P, g, ds, [truth] * k, stream)
        e_ms, r_ms, cnt = kernel_times(P, g, ds, [truth] * k, stream)
        out[prec] = {"events_evals_per_s": n * k / el, "ms_per_eval": el / k * 1e3,
                     "kernel_ms": e_ms, "reduce_ms": r_ms}
        ds.free()
    ncols = len(spec["obs"])
    bytes32 = 4.0 * ncols * n
    k_ms = out["fp32"]["kernel_ms"]
    work = WORK.get(args.workload, {"bound": "hbm"})
    if work["bound"] == "alu":
        tf = work["flops"] * n / (k_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP32_PEAK_TFLOPS, "traffic": None, "algorithmic_flops_per_event": work["flops"],
                "fp64_path": {"achieved": work["flops"] * n / (out["fp64"]["kernel_ms"] * 1e-3) / 1e12,
                              "peak": FP64_PEAK_TFLOPS}}
    else:
        roof = {"bound": "hbm", "achieved": bytes32 / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": bytes32 / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None}
    roof["kernel_ms"] = k_ms
    # device copy of the same footprint (read + write bytes over time)
    a = torch.empty(int(bytes32), dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    out["copy_same_footprint_gbs"] = 2.0 * bytes32 * 20 / (time.perf_counter() - t0) / 1e9
    del a, b
    res = {
        "metric": "events x NLL+grad evaluations per second", "value": out["fp32"]["events_evals_per_s"],
        "unit": "events*evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": out["fp32"]["ms_per_eval"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": spec["name"] + ("_large" if args.workload in large else ""), "n_events": n},
        "roofline": roof,
        "cpu_baseline": None, "extra": out,
    }
    print(json.dumps(res))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1311_1753_amd as P
    import synthgen as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel(), "launches": 5}))
        return
    if args.workload != "c2":
        return other_workload(args, P, S, torch, stream)
    spec = S.C2
    n = spec["n_events"]
    t_gen = time.perf_counter()
    data = S.gen_c2()
    log("generated %d events in %.1f s" % (n, time.perf_counter() - t_gen))
    g = P.Graph.from_spec(spec)
    ds32 = P.Dataset(g, data, "fp32", stream)
    ds64 = P.Dataset(g, data, "fp64", stream)
    truth = g.theta(spec["truth"])
    rng = np.random.default_rng(0)

    # ---------------- settle, warmup, timed region (FP32-eval NLL + gradient)
    n_settle = settle(P, g, ds32, truth, stream, args.settle_s)
    for th in theta_sequence(truth, args.warmup, rng):
        P.nll_grad(g, ds32, th, stream)
    thetas = theta_sequence(truth, args.steps, rng)
    torch.cuda.synchronize()
    el = time_evals(P, g, ds32, thetas, stream)
    ms_step = el / args.steps * 1e3
    value = n * args.steps / el
    # kernel durations: the same evaluations again, every launch timed
    k_ms, r_ms, ncalls = kernel_times(P, g, ds32, thetas if args.steps >= 200 else
                                      theta_sequence(truth, 200, rng), stream)
    alg_bytes = 4.0 * n
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    log("fp32 nll+grad: %.4f ms/step, kernel %.4f ms, reduce %.4f ms" % (ms_step, k_ms, r_ms))

    extra = {"settle_evaluations": n_settle, "kernel_ms_launches": ncalls, "reduce_ms": r_ms}
    # ---------------- latency distribution of single FP32 evaluations
    lat = []
    for th in theta_sequence(truth, 500, rng):
        t1 = time.perf_counter()
        P.nll_grad(g, ds32, th, stream)
        lat.append(time.perf_counter() - t1)
    lat = np.array(lat) * 1e6
    extra["fp32_nll_grad_latency_us"] = {"median": float(np.median(lat)), "p99": float(np.percentile(lat, 99)),
                                         "n": int(lat.size)}
    # ---------------- FP64 analytic and FP64 NLL-only (numerical-gradient path)
    k64 = max(200, args.steps // 10)
    th64 = theta_sequence(truth, k64, rng)
    settle(P, g, ds64, truth, stream, args.settle_s / 2)
    el64 = time_evals(P, g, ds64, th64, stream)
    el64n = time_evals(P, g, ds64, th64, stream, grad=False)
    e64, _, _ = kernel_times(P, g, ds64, th64, stream)
    e64n, _, _ = kernel_times(P, g, ds64, th64, stream, grad=False)
    n_free = int(g.free_mask().sum())
    fp64_value = n * k64 / el64
    fp64_num_value = n * k64 / (el64n * (1 + 2 * n_free))
    extra["fp64_nll_grad_kernel_ms"] = e64
    extra["fp64_nll_only_kernel_ms"] = e64n

    # ---------------- whole fits (minimiser + every evaluation)
    if not args.no_fits:
        t32, r32 = fit_timing(P, g, ds32, stream, "analytic", 3)
        t64, r64 = fit_timing(P, g, ds64, stream, "analytic", 3)
        t64n, r64n = fit_timing(P, g, ds64, stream, "numerical", 2)
        sig = r64["errors"]
        extra["fit_s"] = {"fp32_analytic": t32, "fp64_analytic": t64, "fp64_numerical": t64n}
        extra["fit_evals"] = {"fp32_analytic": r32["n_eval"], "fp64_analytic": r64["n_eval"],
                              "fp64_numerical": r64n["n_eval"]}
        extra["fits_per_s_fp32_analytic"] = 1.0 / t32
        extra["fits_per_s_fp64_numerical"] = 1.0 / t64n
        extra["fp32_fit_dtheta_over_sigma_vs_fp64"] = float(np.max(np.abs(r32["theta"] - r64["theta"]) / sig))

    # ---------------- binned fits: the same 10^7 events in 2000 bins
    if not args.no_fits:
        counts, edges = np.histogram(data["x"], bins=2000, range=(5.2, 5.3))
        cen = {"x": 0.5 * (edges[1:] + edges[:-1])}
        binned = {}
        for metric in ("bnll", "chi2"):
            for prec in ("fp32", "fp64"):
                bd = P.Dataset.binned(g, cen, counts.astype(np.float64), edges[1] - edges[0], metric, prec, stream)
                for _ in range(10):
                    P.nll_grad(g, bd, truth, stream)
                k = 500
                t1 = time.perf_counter()
                for th in theta_sequence(truth, k, rng):
                    P.nll_grad(g, bd, th, stream)
                e_us = (time.perf_counter() - t1) / k * 1e6
                t1 = time.perf_counter()
                rb = P.fit(g, bd, stream=stream)
                binned["%s_%s" % (metric, prec)] = {"us_per_eval": e_us, "fit_ms": (time.perf_counter() - t1) * 1e3,
                                                     "fit_evals": rb["n_eval"], "status": rb["status"]}
                bd.free()
        extra["binned_2000_bins"] = binned

    # ---------------- serving: stream of toy fits (exponential model)
    if not args.no_serving:
        extra["serving"] = serving_bench(P, S, args.serving_requests)

    # ---------------- oracle on the host
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(spec, data, args.cpu_seconds)
        log("oracle: %.3g events*evals/s on %d threads" % (cpu["value"], cpu["cores"]))
        extra["oracle_other_workloads"] = oracle_timing(P, S, stream, fits=not args.no_oracle_fits)

    out = {
        "metric": "events x NLL+grad evaluations per second",
        "value": value,
        "unit": "events*evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the metric's comparison: the same evaluations on the plain FP64 path
        # (FP64 events and arithmetic), with the analytic gradient and with
        # central differences (1 + 2 x 4 NLL-only evaluations per gradient)
        "fp64_path": {"value": fp64_value, "numerical_grad_value": fp64_num_value,
                      "unit": "events*evals/s", "evals": k64},
        "vs_fp64_analytic": value / fp64_value,
        "vs_fp64_numerical_grad": value / fp64_num_value,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gauss+exp composite, x in [5.2,5.3], 1e7 events, 4 free params, "
                               "FP32-eval NLL+analytic gradient, FP64 compensated accumulation",
                   "n_events": n, "n_free_params": n_free},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch",
                     "kernel": "k_mix<float,2,1,true>", "kernel_ms": k_ms,
                     "kernel_ms_from": "HIP events on every launch of an untimed pass repeating the timed "
                                       "evaluations",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
