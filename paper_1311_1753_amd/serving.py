"""Continuous batching of toy / pseudo-experiment fits.

`BatchEngine` wraps the library's batch engine: up to `max_slots` fits of one
graph run concurrently, every `step()` advances each running fit's minimiser
by one likelihood evaluation, and all of those evaluations share one
graph-captured GPU launch.  Admission is by device memory: the datasets of
running fits may hold at most `hbm_budget_bytes`.

`FitServer` is the request loop: requests arrive over time (each with its own
event sample), are uploaded on a separate thread and stream, admitted in FIFO
order as slots and budget free up, stepped together, and retired as they
converge -- requests that arrive while others are on the GPU join the running
batch at the next step boundary.  Device memory is reserved before an
upload: a request's dataset is put on the device only when the datasets
already there (running and waiting fits) leave room for it within the
budget, so the datasets never hold more than `hbm_budget_bytes`; waiting
requests stay host columns until then.  It records per-request latency
(arrival to result on the host) and overall fits/s.
"""
import collections
import ctypes
import queue
import threading
import time

import numpy as np

from . import _lib
from ._lib import check, lib
from .core import Dataset, _dp, _stream_ptr


class BatchEngine:
    def __init__(self, graph, max_slots=256, hbm_budget_bytes=16 << 30):
        self.graph = graph
        h = ctypes.c_void_p()
        check(lib().batch_create(graph.handle, max_slots, int(hbm_budget_bytes), None, ctypes.byref(h)))
        self._h = h
        self.max_slots = max_slots

    def admit(self, ds, theta0=None, tag=0, max_iter=500, edm_tol=1e-10, want_errors=True):
        """Returns the slot, or None when no slot / budget is free right now."""
        th = np.ascontiguousarray(self.graph.theta() if theta0 is None else theta0, dtype=np.float64)
        o = _lib.hf_fit_opts(max_iter, edm_tol, 0, int(want_errors))
        slot = ctypes.c_int32()
        rc = lib().batch_admit(self._h, ds.handle, _dp(th), ctypes.byref(o), int(tag), ctypes.byref(slot))
        if rc in (_lib.HF_E_FULL, _lib.HF_E_BUDGET):
            return None
        check(rc)
        return slot.value

    def step(self):
        a, d = ctypes.c_int32(), ctypes.c_int32()
        check(lib().batch_step(self._h, ctypes.byref(a), ctypes.byref(d)))
        return a.value, d.value

    def poll(self, max_n=None):
        max_n = self.max_slots if max_n is None else max_n
        npar = self.graph.n_par
        tags = (ctypes.c_int64 * max_n)()
        st = np.zeros(max_n, dtype=np.int32)
        th = np.zeros((max_n, npar))
        er = np.zeros((max_n, npar))
        nll = np.zeros(max_n)
        ne = np.zeros(max_n, dtype=np.int32)
        i32 = ctypes.POINTER(ctypes.c_int32)
        k = check(lib().batch_poll(self._h, max_n, tags, st.ctypes.data_as(i32), _dp(th), _dp(er), _dp(nll),
                                   ne.ctypes.data_as(i32)))
        return [{"tag": tags[i], "status": _lib.STATUS_NAMES.get(int(st[i]), str(st[i])), "theta": th[i].copy(),
                 "errors": er[i].copy(), "nll": nll[i], "n_eval": int(ne[i])} for i in range(k)]

    def cancel(self, tag):
        check(lib().batch_cancel(self._h, int(tag)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FitServer:
    """FIFO request loop over a BatchEngine with a background upload thread."""

    def __init__(self, graph, precision="fp32", max_slots=256, hbm_budget_bytes=16 << 30, upload_stream=None):
        self.graph = graph
        self.precision = precision
        self.budget = int(hbm_budget_bytes)
        self.engine = BatchEngine(graph, max_slots, hbm_budget_bytes)
        self.upload_stream = upload_stream

    def run(self, requests, columns_of, theta0_of=None, realtime=True, max_iter=500, edm_tol=1e-10,
            dataset_of=None):
        """Serves `requests` (dicts with 'id' and 'arrival_s', in arrival order).

        columns_of(req) -> event columns, uploaded from the host; or
        dataset_of(req, stream) -> Dataset made on the device (e.g. a toy
        drawn with Dataset.generate), columns_of then unused; either way
        the event count (the columns' length) gives the device bytes
        reserved before the dataset is made (req["n"] when the columns are
        not given).
        theta0_of(req) -> start values.  realtime=False submits every request
        at t = 0 (closed loop).  Returns (results by id, summary)."""
        reqs = sorted(requests, key=lambda r: r["arrival_s"])
        arrivals = {r["id"]: (r["arrival_s"] if realtime else 0.0) for r in reqs}
        ready = queue.Queue()
        t0 = time.perf_counter()
        stop = threading.Event()
        errors = []
        # device bytes of the datasets made and not yet freed (waiting and
        # running fits), guarded by `room`
        room = threading.Condition()
        held = {"bytes": 0, "peak": 0}

        def reserve(nbytes):
            if nbytes > self.budget:
                raise ValueError("a request's dataset (%d bytes) exceeds the whole budget (%d bytes)"
                                 % (nbytes, self.budget))
            with room:
                while held["bytes"] + nbytes > self.budget and not stop.is_set():
                    room.wait(timeout=0.5)
                held["bytes"] += nbytes
                held["peak"] = max(held["peak"], held["bytes"])

        def release(nbytes):
            with room:
                held["bytes"] -= nbytes
                room.notify_all()

        def uploader():
            try:
                for r in reqs:
                    wait = arrivals[r["id"]] - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                    if stop.is_set():
                        return
                    cols = None
                    if dataset_of is not None:
                        n = int(r["n"])
                    else:
                        cols = columns_of(r)
                        n = len(next(iter(cols.values())))
                    need = self.graph.dataset_bytes(n, self.precision)
                    reserve(need)
                    if stop.is_set():
                        release(need)
                        return
                    if dataset_of is not None:
                        ds = dataset_of(r, self.upload_stream)
                    else:
                        ds = Dataset(self.graph, cols, self.precision, self.upload_stream)
                    if ds.device_bytes != need:
                        release(need)
                        reserve(ds.device_bytes)
                    ready.put((r, ds))
            except Exception as e:  # surfaced by the main loop
                errors.append(e)
            finally:
                ready.put(None)

        th = threading.Thread(target=uploader, daemon=True)
        th.start()
        waiting = collections.deque()
        live = {}
        results = {}
        upload_done = False
        steps = 0
        eng = self.engine
        try:
            while True:
                # collect uploaded requests
                while True:
                    try:
                        item = ready.get_nowait() if (waiting or live or upload_done) else ready.get(timeout=0.5)
                    except queue.Empty:
                        break
                    if item is None:
                        upload_done = True
                        break
                    waiting.append(item)
                if errors:
                    raise errors[0]
                # FIFO admission while slots and budget allow
                while waiting:
                    r, ds = waiting[0]
                    th0 = theta0_of(r) if theta0_of else None
                    slot = eng.admit(ds, th0, tag=r["id"], max_iter=max_iter, edm_tol=edm_tol)
                    if slot is None:
                        break
                    waiting.popleft()
                    live[r["id"]] = (r, ds, time.perf_counter() - t0)
                if live:
                    eng.step()
                    steps += 1
                    for res in eng.poll():
                        r, ds, t_adm = live.pop(res["tag"])
                        t_done = time.perf_counter() - t0
                        nbytes = ds.device_bytes
                        ds.free()
                        release(nbytes)
                        res.update({"arrival_s": arrivals[r["id"]], "admit_s": t_adm, "done_s": t_done,
                                    "latency_s": t_done - arrivals[r["id"]], "n_events": ds.n})
                        results[r["id"]] = res
                elif upload_done and not waiting:
                    break
        finally:
            stop.set()
            with room:
                room.notify_all()
            th.join(timeout=60)
        lat = np.array([v["latency_s"] for v in results.values()])
        done = np.array([v["done_s"] for v in results.values()])
        first = min(arrivals.values())
        span = done.max() - first if done.size else float("nan")
        summary = {"n": len(results), "steps": steps, "makespan_s": float(span),
                   "fits_per_s": len(results) / span if span > 0 else float("nan"),
                   "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else float("nan"),
                   "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else float("nan"),
                   "statuses": dict(collections.Counter(v["status"] for v in results.values())),
                   "peak_dataset_bytes": held["peak"], "budget_bytes": self.budget}
        return results, summary

    def close(self):
        self.engine.close()


def serve_one_at_a_time(graph, requests, columns_of, theta0_of=None, precision="fp64", grad_mode="numerical",
                        stream=None, realtime=False):
    """Baseline: each request uploaded and fitted alone, in arrival order.

    realtime=False (closed loop): the requests run back to back from t = 0;
    fits/s = requests / wall time, latencies = finish - arrival with every
    arrival at 0 (their queueing behind earlier requests included).
    realtime=True (open loop): a request starts at its arrival time (or when
    the previous one finishes, if later), as a single-server queue run on
    the wall clock; latency = finish - arrival, measured."""
    from .core import fit
    reqs = sorted(requests, key=lambda r: r["arrival_s"])
    service = []
    results = {}
    lat = []
    t_start = time.perf_counter()
    for r in reqs:
        if realtime:
            wait = t_start + r["arrival_s"] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
        t0 = time.perf_counter()
        ds = Dataset(graph, columns_of(r), precision, stream)
        res = fit(graph, ds, theta0_of(r) if theta0_of else None, grad_mode=grad_mode, stream=stream)
        ds.free()
        t1 = time.perf_counter()
        service.append(t1 - t0)
        lat.append(t1 - (t_start + r["arrival_s"]) if realtime else t1 - t_start)
        results[r["id"]] = res
    span = time.perf_counter() - t_start
    lat = np.array(lat)
    return results, {"n": len(reqs), "mode": "open loop (wall clock)" if realtime else "closed loop",
                     "fits_per_s": len(reqs) / span, "fits_per_s_saturated": len(reqs) / float(np.sum(service)),
                     "makespan_s": span, "p50_latency_s": float(np.percentile(lat, 50)),
                     "p99_latency_s": float(np.percentile(lat, 99)),
                     "mean_service_s": float(np.mean(service))}
